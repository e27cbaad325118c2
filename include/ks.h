/*
 * ks.h — C ABI of the MI355X (gfx950) Kohn-Sham direct-minimisation library.
 *
 * The library minimises the discretised Kohn-Sham total energy over the Stiefel
 * manifold, min E(X) s.t. X^T X = I_p (Zhang, Zhu, Wen, Zhou, "Gradient type
 * optimization methods for electronic structure calculations", Section 3 eq. (opt)),
 * without linear eigensolves.  Every step on the data path runs in HIP kernels on
 * the device; the host side only orders launches and reads back a few scalars.
 *
 * Conventions shared by all calls
 * -------------------------------
 * - Grid.  A uniform interior grid of nx*ny*nz points with spacing h; point (i,j,k)
 *   (0-based) sits at box_lo + ((i+1)h, (j+1)h, (k+1)h) and has linear index
 *   g = i + nx*(j + ny*k).  Values outside the interior grid are zero (Dirichlet).
 * - Orbital blocks (X, G, gradE) are device pointers to n x p matrices stored
 *   grid-major: element (g, i) at [g*ld + i], ld >= p given in the descriptor.
 *   The element type is double (KS_PREC_FP64) or float (KS_PREC_FP32 and
 *   KS_PREC_MIXED_BF16).  Density and potentials are double device vectors of n.
 * - Energy units are Hartree, lengths bohr.  Orbitals are normalised by
 *   X^T X = I, i.e. phi_i(r_g) = X_gi h^{-3/2}; the density is
 *   rho_g = (f/h^3) sum_i X_gi^2 with occupation f per orbital.
 * - Finite elements (KS_DISC_Q1).  The grid points are the nodes of trilinear elements
 *   on cubes of side h (Section 2.3, the finite-element form with the mass matrix B).
 *   Orbitals are nodal coefficients with X^T B X = I, B = M x M x M and stiffness
 *   A = K x M x M + M x K x M + M x M x K from the 1D linear-element matrices
 *   K = (1/h) tridiag(-1, 2, -1), M = (h/6) tridiag(1, 4, 1).  Potential terms use nodal
 *   quadrature: rho_k = f sum_i X_ki^2, A V_H = 4 pi h^3 rho, and
 *   E_X = 2f [ (1/2) A X + h^3 Diag(V_ext + V_H + v_x) X ].  The manifold is handled in
 *   the B metric (Section 3 with Y = B^{1/2} X, as eq. (OFDFT-y) does for p = 1):
 *   gradE = B^{-1} G - X G^T X, ||gradE||^2 = tr(gradE^T B gradE), the QR retraction
 *   factors Y^T B Y, and ks_energy reports ||X^T B X - I||_F.  Only the QR retraction is
 *   built for this form, and each axis holds at most 128 nodes.
 * - Memory.  The caller owns every device buffer, including the workspace handed
 *   to ks_create_system; the library never allocates or frees device memory.
 *   The library allocates a 9 KiB pinned host buffer per system for scalar
 *   read-back (freed by ks_destroy_system); the device writes the records of a line-search
 *   trial into it directly.
 * - Streams.  Work of a system is issued on the HIP stream given at creation.  All
 *   calls below return after that stream has finished the call's work
 *   (synchronous), unless stated otherwise.  One system handle must not be used
 *   from two threads at once; different handles are independent.
 * - Errors.  Every int-returning call returns KS_OK (0) or a negative KS_E_*
 *   code; no exception crosses the ABI.  ks_last_error() gives a message.
 */
#ifndef KS_H
#define KS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------------------- */
#define KS_OK 0
#define KS_E_INVAL (-1)          /* bad argument or descriptor                            */
#define KS_E_NOMEM (-2)          /* workspace smaller than ks_workspace_bytes()           */
#define KS_E_HIP (-3)            /* a HIP runtime call failed                             */
#define KS_E_NOT_SPD (-4)        /* Cholesky breakdown (Y^T Y or X^T X not positive def.) */
#define KS_E_SINGULAR (-5)       /* singular Sherman-Morrison-Woodbury system (WY)        */
#define KS_E_NONFINITE (-6)      /* NaN or Inf in an energy, gradient or step             */
#define KS_E_NOT_CONVERGED (-7)  /* ks_minimize stopped at max_iter                       */
#define KS_E_UNSUPPORTED (-8)    /* combination not implemented                           */

/* ---- enums ------------------------------------------------------------------------- */
#define KS_DISC_FD7 0            /* 7-point finite differences (Section 2.3)              */
#define KS_DISC_Q1 1             /* trilinear finite elements, B-orthonormality           */

#define KS_PREC_FP64 0           /* everything in double                                  */
#define KS_PREC_FP32 1           /* X, G stored/applied in float; reductions in double    */
#define KS_PREC_MIXED_BF16 2     /* as FP32; X^T G of blocks wider than 64 columns on bf16
                                    matrix cores with fp32 sums.  X^T G only sets the
                                    direction D = G - X (X^T G)^T; the Gram blocks the
                                    retraction factors (X^T X, X^T D, D^T D) are products
                                    of the stored blocks, so X stays orthonormal to the
                                    float rounding of its entries.  The gradient norm then
                                    carries the bf16 error of X^T G: stop on
                                    energy_target.  Not accepted by the server.          */
#define KS_PREC_FP32_MFMA 3      /* as FP32, and the block combines of blocks wider than
                                    64 columns (retraction X A + Y B, direction
                                    G + X W) run on the fp32 matrix cores: weights
                                    rounded to float, fp32 sums over chains of 64
                                    contraction indices, FP64 across chains, so an entry
                                    is off by at most (64 + 4) 2^-24 of the sum of
                                    |products| before its float store.  Gram blocks as
                                    in FP32.  Not accepted by the server.                */

#define KS_TERM_EXT 1            /* external (nuclear) potential                          */
#define KS_TERM_HARTREE 2        /* Hartree potential                                     */
#define KS_TERM_XC 4             /* Slater exchange                                       */
#define KS_TERM_ALL 7            /* external + Hartree + Slater exchange                  */
#define KS_TERM_CORR 8           /* LDA correlation, Perdew-Zunger (1981) parametrisation
                                    of the Ceperley-Alder electron gas (unpolarised); with
                                    KS_TERM_XC the full LDA of Section 4.  Its energy is
                                    reported in ks_energy.xc with the exchange            */
#define KS_TERM_TF 16            /* Thomas-Fermi kinetic energy C_TF int rho^{5/3}, C_TF =
                                    (3/10)(3 pi^2)^{2/3} (Section 2.2 eq. (TFW)); reported in
                                    ks_energy.kinetic.  With p = 1, occupation N (electrons)
                                    and kinetic_scale mu, the run is the orbital-free TFW
                                    model of eq. (OFeng): the kinetic term (mu f/2) X^T L X
                                    is then the von Weizsaecker energy mu T_vW of
                                    rho = N phi^2, and the constraint is int phi^2 = 1     */

#define KS_VEXT_ERF 0            /* sum_a -Z_a erf(|r - R_a|/rc)/|r - R_a|                */
#define KS_VEXT_GNH 1            /* Goodwin-Needs-Heine local pseudopotential of Section
                                    4.2 (R = 1.15, R_c = 3.5, A = 0.1107), the
                                    electron-ion attraction (tends to -Z/r)               */

/* Boundary values of the Hartree potential (Section 2.3 poses the Poisson problem on the
 * box): zero Dirichlet (a grounded box), or the monopole values Q/|r_b - c| of the electron
 * count Q = f p about the nuclear-charge centre c, which a finite charged cluster needs for
 * free-space electrostatics.  The monopole option adds the fixed harmonic potential V_bc
 * (Q times the harmonic extension of 1/|r_b - c|, computed once at creation with the
 * system's Hartree solver) to V_eff, and h^3 sum rho V_bc - (1/2) Q V_bc(c) to E_H; E_X
 * remains the exact derivative of the reported energy. */
#define KS_HBC_ZERO 0
#define KS_HBC_MONOPOLE 1

#define KS_HARTREE_CG 0          /* plain conjugate gradients, warm started               */
#define KS_HARTREE_PCG_FD 1      /* CG preconditioned by the exact fast diagonalisation   */

#define KS_QR 0                  /* retraction eq. (QR) by Cholesky QR (Alg. 2)           */
#define KS_WY 1                  /* Cayley retraction eq. (WY3)                           */

#define KS_BB_ALT 0              /* tau_{k,1} on odd k, tau_{k,2} on even k               */
#define KS_BB1 1
#define KS_BB2 2

#define KS_STOP_NONE 0
#define KS_STOP_GRAD 1           /* ||grad E||_F <= eps_g                                  */
#define KS_STOP_STAGNATION 2     /* mean of last three relative energy changes < tol      */
#define KS_STOP_MAXIT 3
#define KS_STOP_ERROR 4
#define KS_STOP_ENERGY 5         /* an accepted energy reached energy_target               */

/* ---- descriptors ------------------------------------------------------------------- */
typedef struct ks_system_desc {
  int disc;                /* KS_DISC_*                                                   */
  int nx, ny, nz;          /* interior points per axis (>= 1)                             */
  double h;                /* grid spacing, bohr (> 0)                                    */
  double box_lo[3];        /* box corner: point (i,j,k) sits at box_lo + (i+1, j+1, k+1) h */
  int p;                   /* orbitals: 1 <= p <= 512 (FD7), 1 <= p <= 128 (Q1)          */
  int ld;                  /* row stride of X/G/gradE in elements; 0 means p              */
  double occupation;       /* f, electrons per orbital (2 = closed shell)                 */
  int n_nuclei;            /* M >= 0                                                      */
  const double* R;         /* host, 3*M coordinates (x,y,z per nucleus); copied           */
  const double* Z;         /* host, M charges; copied                                     */
  double rc;               /* erf smoothing radius of the nuclear potential (> 0)         */
  int terms;               /* KS_TERM_* bit mask                                          */
  const double* v_ext_override; /* host, n values replacing the nuclear potential, or NULL */
  int precision;           /* KS_PREC_*                                                   */
  int hartree_solver;      /* KS_HARTREE_*                                                */
  double hartree_tol;      /* relative residual ||r||/||4 pi rho||; <= 0 means 1e-13.
                              A KS_HARTREE_PCG_FD solve whose residual stops falling
                              (3 iterations without a 4x decrease: the rounding floor,
                              about eps cond(L)) also ends once it is within 100x of it */
  int hartree_maxit;       /* <= 0 means 5000                                             */
  double kinetic_scale;    /* mu: H = (mu/2) L + V_eff (the von Weizsaecker weight of
                              eq. (TFW) for orbital-free runs); <= 0 means 1              */
  int vext_kind;           /* KS_VEXT_* form of the nuclear potential                     */
  int hartree_bc;          /* KS_HBC_* boundary values of the Hartree potential           */
} ks_system_desc;

typedef struct ks_energy {
  double total;            /* E_KS, eq. (EKS) in the discrete form of Section 2.3         */
  double kinetic;          /* (mu f/2) tr(X^T L X), L = -Laplacian_h (plus the
                              Thomas-Fermi energy with KS_TERM_TF)                        */
  double external;         /* h^3 sum V_ext rho                                           */
  double hartree;          /* (h^3/2) rho^T V_H (+ the monopole boundary terms)           */
  double xc;               /* h^3 sum rho (eps_x(rho) + eps_c(rho) with KS_TERM_CORR)      */
  double nuclear;          /* E_II                                                        */
  double grad_norm;        /* ||G - X G^T X||_F with G = E_X                              */
  double orth_error;       /* ||X^T X - I||_F                                             */
  int hartree_iters;       /* CG iterations of this evaluation                            */
  double hartree_relres;   /* final relative residual                                     */
} ks_energy;

typedef struct ks_opt_params {
  double tau0;             /* first step and fallback for an unusable BB value (1e-3)     */
  double rho1;             /* Armijo constant in eq. (NMLS-Armijo) (1e-4)                 */
  double delta;            /* backtracking factor (0.1)                                   */
  double eta;              /* weight of the reference value C_k (0.85)                    */
  double eps_g;            /* stop when ||grad E||_F <= eps_g (1e-6, Section 4.1)         */
  int max_iter;            /* (10000)                                                     */
  int bb_rule;             /* KS_BB_*                                                     */
  int retraction;          /* KS_QR or KS_WY                                              */
  double tau_min, tau_max; /* clamp of the BB value (1e-20, 1e20)                         */
  int h_max;               /* backtracks before a trial is accepted anyway (20)           */
  double reorth_tol;       /* WY: re-orthonormalise when ||X^T X - I||_F > tol (1e-12)    */
  double stagnation_tol;   /* stop when mean(df_k, df_k-1, df_k-2) < tol (1e-13); 0 = off */
  int reorth_every;        /* > 0: every reorth_every accepted iterations, X <- X R^{-1}
                              with X^T X = R^T R (X^T B X for Q1) formed from the stored
                              X in FP64 (Cholesky QR, Alg. 2), the point evaluated again
                              and the nonmonotone reference restarted there (C = E,
                              Q = 1).  For reduced-precision storage (0 = never)          */
  double energy_target;    /* stop (KS_STOP_ENERGY) once an accepted energy is <= this;
                              -HUGE_VAL = off (default).  The reduced-precision modes
                              stop on it: their gradient stalls at the float resolution
                              of X above eps_g                                            */
} ks_opt_params;

typedef struct ks_result {
  int iters;               /* accepted iterations k                                       */
  int nfe;                 /* energy evaluations                                          */
  int backtracks;          /* rejected trial steps                                        */
  int ls_fail;             /* trials accepted after h_max reductions without Armijo       */
  int reorths;             /* WY re-orthonormalisations                                   */
  int stop_reason;         /* KS_STOP_*                                                   */
  double energy;           /* final E                                                     */
  double grad_norm;        /* final ||grad E||_F                                          */
  ks_energy terms;         /* final energy terms                                          */
  double seconds;          /* wall time of the call                                       */
  long long hartree_iters_total;
} ks_result;

/* Progress of a run after a step of the per-iteration calls below. */
typedef struct ks_iter_info {
  int k;                   /* accepted iterations so far                                  */
  int nfe;                 /* energy evaluations so far                                   */
  int backtracks;          /* rejected trial steps so far                                 */
  int stop_reason;         /* KS_STOP_* (KS_STOP_NONE while the run goes on)              */
  double energy;           /* E(X_k)                                                      */
  double grad_norm;        /* ||grad E(X_k)||_F (the B-norm for KS_DISC_Q1)               */
  double tau;              /* step of the last accepted trial (0 before the first)        */
  double C;                /* reference value C_k of eq. (NMLS-Armijo)                    */
} ks_iter_info;

/* Phases of the device timeline measured by the optional timers (ks_enable_timers).
 * The single-kernel phases bracket exactly one kernel per occurrence. */
#define KS_PH_HARTREE 0          /* one Hartree solve (all CG kernels of it)              */
#define KS_PH_XC 1               /* exchange and effective potential (one kernel)         */
#define KS_PH_HAMILTONIAN 2      /* G = 2f H X with energy partials (one kernel; Q1: and
                                    B X in the same kernel)                               */
#define KS_PH_GRAM 3             /* Gram blocks of [X, G] or [X, D] (one kernel)          */
#define KS_PH_GRADIENT 4         /* grad E = G - X G^T X with BB sums (one kernel; Q1: the
                                    B^{-1} G sweeps, then grad E and B grad E)            */
#define KS_PH_RETRACT 5          /* X+ = X A + Y B with fused density (one kernel)        */
#define KS_PH_SMALL 6            /* reductions, small dense factors, line-search logic    */
#define KS_PH_DENSITY 7          /* stand-alone density (first evaluation)                */
#define KS_NPHASES 8

typedef struct ks_phase_times {
  double ms[KS_NPHASES];        /* accumulated device time per phase, milliseconds       */
  long long count[KS_NPHASES];  /* occurrences                                           */
} ks_phase_times;

/* Launch shapes chosen by ks_autotune (KS_TUNE_AUTO: the built-in rule applies). */
#define KS_TUNE_AUTO (-99)
typedef struct ks_tune_info {
  int fd_plane_mode;   /* plane-transform mode of the fast-diagonalisation Hartree solver:
                          2 whole plane per block, 1 16-column strips with S_y staged,
                          0 strips, -1 strips with S_x read from L2; KS_TUNE_AUTO if not
                          tuned (no fast-diagonalisation solver)                          */
  int hx_zrun;         /* z-planes per work item of the Hamiltonian with fused Gram tiles
                          (8 or 16), KS_TUNE_AUTO if not tuned (that kernel is used at
                          p = 32 on the 7-point grid only)                                */
  int cached;          /* 1: the choice came from the process-wide cache                 */
  int n_fd, n_hx;      /* candidates timed (0 when cached)                               */
  int fd_modes[4];     /* candidate modes and their mean time per solve, microseconds    */
  double fd_us[4];
  int hx_zruns[2];     /* candidate runs and their mean time per launch, microseconds    */
  double hx_us[2];
} ks_tune_info;

typedef struct ks_system ks_system;

/* ---- sizing and lifecycle -------------------------------------------------------------- */

/* Device bytes ks_create_system needs for this descriptor (all resident state of one
 * system: potentials, density, CG vectors, the current/trial orbital blocks and their
 * gradients, Gram and small dense buffers, reduction partials).  0 if invalid. */
size_t ks_workspace_bytes(const ks_system_desc* d);

/* Creates a system: validates d, carves the caller's device workspace (ws_bytes >=
 * ks_workspace_bytes(d), 256-byte aligned), copies nuclei to the device, and computes
 * V_ext and E_II there (setup of Section 2.1 eq. (EKS)).  hip_stream is a hipStream_t
 * (NULL = default stream).  On success *out receives the handle.  Errors: KS_E_INVAL
 * (also when the first or last byte of the needed workspace is not memory the HIP runtime
 * reports as device or managed memory; nothing is launched then), KS_E_NOMEM, KS_E_HIP,
 * KS_E_UNSUPPORTED. */
int ks_create_system(const ks_system_desc* d, void* dev_workspace, size_t ws_bytes,
                     void* hip_stream, ks_system** out);

/* Releases the handle and its pinned host buffer (not the caller's workspace). */
void ks_destroy_system(ks_system* s);

/* Default optimiser parameters (values in the comments of ks_opt_params). */
void ks_default_params(ks_opt_params* o);

const char* ks_status_string(int code);
const char* ks_last_error(const ks_system* s);

/* ---- the method --------------------------------------------------------------------- */

/* Energy and partial derivative at X (Section 2.3 eq. (partial deriv)):
 *   G = E_X = 2f [ (1/2) L X + Diag(V_ext + V_H + v_x) X ],
 *   gradE = G - X G^T X (Section 3 eq. (def-nablaE)).
 * X, G, gradE: device n x ld blocks; G and gradE may be NULL (not written).  out (host)
 * receives the energy terms, ||gradE||_F and ||X^T X - I||_F.  The Hartree solve is
 * warm-started from the potential of the previous call on this system, and its result
 * becomes the next warm start.  Errors: KS_E_INVAL, KS_E_HIP, KS_E_NONFINITE. */
int ks_energy_grad(ks_system* s, const void* X, void* G, void* gradE, ks_energy* out);

/* One retraction from X along the descent direction built from G = E_X:
 *   KS_QR: X_out = qr(X - tau gradE) by Cholesky QR (eq. (QR), Alg. 2);
 *   KS_WY: X_out = X - tau U (I + tau/2 V^T U)^{-1} V^T X, U = [G, X], V = [X, -G]
 *          (eq. (WY3)).
 * X, G, X_out: device n x ld blocks; X_out must not alias X or G.  Errors: KS_E_INVAL,
 * KS_E_NOT_SPD (Cholesky breakdown), KS_E_SINGULAR (zero pivot in the 2p x 2p LU),
 * KS_E_NONFINITE, KS_E_HIP. */
int ks_retract(ks_system* s, const void* X, const void* G, double tau, int kind,
               void* X_out);

/* Alg. 3 from X_inout (orthonormal columns expected; for KS_DISC_Q1 any full-rank block,
 * which is first B-orthonormalised by Cholesky QR in the B metric) with BB steps (eq. (bb-1)) and the
 * nonmonotone Armijo search (eq. (NMLS-Armijo)); on return X_inout holds the last
 * accepted iterate and *r (host) the statistics.  The first Hartree solve of a run
 * starts from V_H = 0, so the result depends only on X_inout and the parameters.  o may be NULL for defaults.  Returns
 * KS_OK when the gradient or stagnation test stopped the run, KS_E_NOT_CONVERGED at
 * max_iter (r filled), or an error code. */
int ks_minimize(ks_system* s, void* X_inout, const ks_opt_params* o, ks_result* r);

/* Runs ks_minimize on count (1..16) systems in lockstep: each kernel of a trial step is one
 * launch for all of them (every system reads its own argument record and keeps the block
 * partition of its lone run), so each result equals that system's lone ks_minimize bit for
 * bit while small systems share the launch cost.  Requires the finite-difference form,
 * the KS_HARTREE_PCG_FD solver with the Hartree term, the QR retraction, p <= 32 and
 * timers off; systems of either storage precision may be mixed.  The launches go to the
 * first system's stream.  r[i] and codes[i] (host, either may be NULL) receive each
 * system's statistics and ks_minimize return code (KS_E_UNSUPPORTED for a system outside
 * these limits).  Returns KS_OK, or the first error other than KS_E_NOT_CONVERGED. */
int ks_minimize_batch(ks_system* const* sys, int count, void* const* X_inout,
                      const ks_opt_params* o, ks_result* r, int* codes);

/* ---- Alg. 3 one iteration at a time ------------------------------------------------------
 * The loop of ks_minimize opened up: ks_minimize_begin does its set-up and first
 * evaluation, ks_minimize_step one iteration of Alg. 3 (trial steps until one satisfies
 * eq. (NMLS-Armijo) or the run stops), ks_minimize_end its finish.  The three calls run
 * exactly the kernels and decisions of ks_minimize, so begin, any number of steps and end
 * give ks_minimize's result bit for bit.  The run's state (the current iterate, its
 * gradient and Gram blocks, the Hartree warm start, the line-search record C_k, Q_k, tau,
 * and the counters) stays in the system's workspace between calls; ks_get_state copies it
 * out and ks_set_state puts it back, on the same or another system of the same
 * descriptor, so that a run resumed from a saved state continues bit for bit. */

/* Starts a run from X0 (device n x ld block, as for ks_minimize; only read).  info (host,
 * nullable) receives k = 0 and the first energy.  Errors as ks_minimize. */
int ks_minimize_begin(ks_system* s, const void* X0, const ks_opt_params* o,
                      ks_iter_info* info);

/* One iteration: trial steps until one is accepted or a stopping rule fires; a stopped
 * run returns at once.  info (host, nullable) receives the progress.  Errors: KS_E_INVAL
 * (no run in progress), the device errors of ks_minimize (the run is then over). */
int ks_minimize_step(ks_system* s, ks_iter_info* info);

/* Ends the run: X_out (device n x ld block, nullable = not copied) receives the current
 * iterate and r (host, nullable) the statistics, as ks_minimize returns them.  Returns
 * KS_OK, KS_E_NOT_CONVERGED at max_iter, or the run's error. */
int ks_minimize_end(ks_system* s, void* X_out, ks_result* r);

/* Bytes of a saved run state of this system (header plus the device records above). */
size_t ks_state_bytes(ks_system* s);

/* Copies the state of the run in progress into buf (host or device memory of
 * ks_state_bytes(s) bytes, owned by the caller).  Synchronous.  Errors: KS_E_INVAL (no run
 * in progress), KS_E_HIP. */
int ks_get_state(ks_system* s, void* buf);

/* Makes the run saved in buf the run in progress of s (whose descriptor must give the same
 * discretisation, precision, n and p; any run in progress is dropped).  Continue with
 * ks_minimize_step / ks_minimize_end.  Errors: KS_E_INVAL (not a state, or one of another
 * shape), KS_E_HIP. */
int ks_set_state(ks_system* s, const void* buf);

/* One trial step for each listed run in lockstep (1..16 systems, each with a run begun by
 * ks_minimize_begin and inside the limits of ks_minimize_batch; runs that have stopped
 * are skipped): one launch per kernel for all of them, as ks_minimize_batch does, on the
 * first system's stream.  Each run takes the decisions of its lone trial, so stepping the
 * batch to the end gives every member its lone ks_minimize result bit for bit.  info
 * (host, count entries, nullable) receives every member's progress; info[i].k tells
 * whether its trial was accepted.  Errors: KS_E_INVAL, KS_E_UNSUPPORTED (a run outside the
 * limits; nothing is launched), the first member error. */
int ks_batch_step(ks_system* const* sys, int count, ks_iter_info* info);

/* ---- launch-shape autotuning ------------------------------------------------------------
 * Times the candidate launch shapes of two kernels of an evaluation on this system's own
 * buffers (the fast-diagonalisation plane transforms of the Hartree solve, every mode whose
 * LDS fits; the Hamiltonian with fused Gram tiles, 8 or 16 planes per work item) and keeps
 * the fastest for the system when it beats the built-in shape by more than 10% (each
 * candidate's best of three interleaved timing rounds; smaller differences are within the
 * run-to-run spread of these timings and must not flip the choice).  Choices are cached per (grid, p, precision, discretisation,
 * Hartree solver) for the process: a later system of the same key takes them without
 * timing (force = 1 times again).  The shapes change how sums split over blocks, so results
 * can differ from untuned runs in the last bits (a saved state resumes bit for bit only on
 * a handle with the same shapes).  Overwrites the system's Hartree warm start and orbital
 * scratch: call it before a run, not during one.  out (host, nullable) receives the choice
 * and the timings.  Errors: KS_E_INVAL (a run in progress), KS_E_HIP. */
int ks_autotune(ks_system* s, int force, ks_tune_info* out);

/* ---- Alg. 4 with uniform refinement -------------------------------------------------
 * Alg. 4 solves the problem on a sequence of meshes, each level started from the solution
 * of the next coarser one carried over to the finer mesh.  Here every level is the uniform
 * refinement of the one before (the variant of Table 5; no a posteriori marking): same box
 * and nuclei, half the spacing, 2N + 1 interior nodes per axis, so coarse node i is fine
 * node 2i + 1.  Both systems of a pair must share the discretisation, precision, p and
 * occupation. */

/* Carries the coarse block Xc (device n_c x ld_c of `coarse`, only read) over to `fine`:
 * trilinear interpolation of the nodal values (for Q1 elements the same finite-element
 * function, exactly), on the 7-point grid rescaled by 2^{-3/2} (phi = X h^{-3/2}), then
 * Cholesky QR (Alg. 2; in the B metric for elements).  Xf (device n_f x ld_f of `fine`)
 * receives an orthonormal block (X^T X = I, or X^T B X = I).  The coarse stream is
 * synchronised first; the work runs on the fine system's stream and is complete on return.
 * Errors: KS_E_INVAL (not a nested pair, or a run of `fine` in progress), KS_E_NOT_SPD
 * (the carried block is rank deficient), KS_E_HIP. */
int ks_prolong(ks_system* coarse, const void* Xc, ks_system* fine, void* Xf);

/* Alg. 4 over nlev (1..16) nested systems, coarsest first: ks_minimize on level 0 from
 * X[0] (in/out, as for ks_minimize), then for each finer level ks_prolong from the level
 * before into X[i] (device n_i x ld_i, written) and ks_minimize there, all with the
 * parameters o (NULL: defaults).  A level that stops at max_iter still seeds the next.
 * r (host, nlev entries, required) receives every level's statistics.  Returns KS_OK when
 * the finest level converged, KS_E_NOT_CONVERGED when it stopped at max_iter, or the first
 * error (naming its level in ks_last_error of that level's system). */
int ks_minimize_levels(ks_system* const* levels, int nlev, void* const* X,
                       const ks_opt_params* o, ks_result* r);

/* ---- step-level calls (each is one step of ks_energy_grad) -------------------------- */

/* rho (device, n doubles) = (f/h^3) sum_i X_gi^2 (Section 2.3, rho(X) = diag(X X^T)). */
int ks_density(ks_system* s, const void* X, double* rho);

/* Solves L v_h = 4 pi rho (L = -Laplacian_h, zero Dirichlet) with the system's Hartree
 * solver to its tolerance.  rho, v_h: device n doubles; if warm != 0, v_h holds the
 * starting guess on entry.  iters/relres (host, nullable) receive the iteration count
 * and final relative residual.  Errors: KS_E_INVAL, KS_E_NOT_CONVERGED, KS_E_HIP. */
int ks_hartree_solve(ks_system* s, const double* rho, double* v_h, int warm, int* iters,
                     double* relres);

/* Y = H X with H = (1/2) L + Diag(v_eff) (the Hamiltonian of eq. (partial deriv) without
 * the factor 2f).  v_eff: device n doubles, or NULL for the potential of the last
 * ks_energy_grad/ks_minimize evaluation.  X, Y: device n x ld blocks, Y != X. */
int ks_apply_hamiltonian(ks_system* s, const void* X, void* Y, const double* v_eff);

/* Copies (device to device) the nuclear potential V_ext and the last Hartree and
 * effective potentials into the given n-double device buffers (any may be NULL). */
int ks_get_potentials(ks_system* s, double* v_ext, double* v_h, double* v_eff);

/* Gram blocks of two device n x ld blocks A, B: out (device, 3*p*p doubles, row-major
 * p x p each) = [A^T A, A^T B, B^T B].  The tall-skinny products of Section 3, summed in
 * FP64 (KS_PREC_MIXED_BF16 above 64 columns: A^T B in bf16 with fp32 sums). */
int ks_gram(ks_system* s, const void* A, const void* B, double* out);

/* ---- no-allocation variant ------------------------------------------------------------ */

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the Gram blocks of ks_gram without a
 * system handle or workspace.  A, B: device n x ld blocks (double for KS_PREC_FP64, float
 * for KS_PREC_FP32 / KS_PREC_MIXED_BF16; products always in FP64); ld = 0 means p.
 * out (device, 3*p*p doubles, row-major p x p each) = [A^T A, A^T B, B^T B].  The call only
 * enqueues work on hip_stream (NULL = default stream) and returns; it calls no hipMalloc,
 * hipFree or allocating routine.  Its partial products live in one static device array of
 * 12.7 MB per GPU, held until the process ends: limits 1 <= p <= 64, n * ld < 2^31 (at most
 * 128 row chunks).  Calls on one GPU share that array, so calls that can overlap on the
 * device (different streams without ordering between them) race; calls on one stream are
 * ordered.  Errors (the message via ks_last_error(NULL)): KS_E_INVAL for sizes beyond the
 * limits or null pointers, KS_E_HIP. */
int ks_gram_static(const void* A, const void* B, int n, int p, int ld, int precision,
                   double* out, void* hip_stream);

/* ---- serving ---------------------------------------------------------------------------
 * A server solves independent minimisation requests concurrently on one GPU.  It owns no
 * device memory: requests are admitted in arrival order into first-fit regions of the
 * caller's workspace, each sized by ks_workspace_bytes() plus the request's orbital block
 * (admission by HBM footprint).  n_slots worker threads each drive one request at a time
 * on a stream of their own, so requests that arrive while others run are admitted as
 * slots and memory free up and their kernels overlap on the device.  A request's result
 * does not depend on its co-tenants (same kernels, same reduction order as running it
 * alone with ks_minimize). */
typedef struct ks_server ks_server;

typedef struct ks_request {
  int id;                   /* caller's tag, echoed in the completion                     */
  ks_system_desc desc;      /* its host arrays (R, Z, v_ext_override) are copied at submit */
  const void* X0;           /* host n x p start block in the desc's precision; the server
                               keeps every orbital block dense (desc.ld is ignored)       */
  void* X_out;              /* host n x p result block, or NULL                           */
  ks_opt_params params;     /* Alg. 3 parameters                                          */
} ks_request;

typedef struct ks_completion {
  int id;
  int status;               /* ks_minimize's return code, or the admission error          */
  ks_result result;
  double t_submit, t_admit, t_done;  /* seconds since ks_server_create                    */
  size_t bytes;             /* device bytes the request held while it ran                 */
} ks_completion;

/* Creates a server over the caller's device workspace (256-byte aligned) with n_slots
 * (1..64) concurrent workers on the current device.  Errors: KS_E_INVAL (including a
 * workspace that is not device memory of ws_bytes bytes), KS_E_HIP. */
int ks_server_create(void* dev_workspace, size_t ws_bytes, int n_slots, ks_server** out);

/* Creates a server in continuous-batching mode: one engine thread keeps up to max_batch
 * (1..16) requests resident and advances them together, one trial step at a time, with
 * one launch per kernel for all of them (ks_minimize_batch's lockstep runner); between
 * steps it admits queued requests into free regions and places, and retires the ones
 * that stopped.  Requests outside the runner's limits run alone on the engine thread.
 * Results equal lone ks_minimize runs bit for bit.  Errors: KS_E_INVAL (as for
 * ks_server_create), KS_E_HIP. */
int ks_server_create_batched(void* dev_workspace, size_t ws_bytes, int max_batch,
                             ks_server** out);

/* Queues a request (copies X0 and the descriptor's host arrays before returning; X_out
 * must stay valid until the request's completion has been polled).  A request larger
 * than the whole workspace completes at once with status KS_E_NOMEM.  Errors: KS_E_INVAL
 * (null arguments, or a descriptor ks_workspace_bytes rejects: ks_last_error(NULL) on
 * the calling thread says why). */
int ks_server_submit(ks_server* sv, const ks_request* rq);

/* Moves up to max finished requests into out (host); *n_out receives the count. */
int ks_server_poll(ks_server* sv, ks_completion* out, int max, int* n_out);

/* Blocks until every submitted request has completed. */
int ks_server_wait_idle(ks_server* sv);

/* Number of requests queued and running. */
int ks_server_pending(ks_server* sv);

/* Stops the workers after the running requests finish; queued requests are dropped. */
void ks_server_destroy(ks_server* sv);

/* ---- launch replay ---------------------------------------------------------------------
 * With graphs on, ks_minimize records its trial step (retraction factor and combine,
 * energy/gradient evaluation, line-search judgement) once per slot parity into a HIP
 * graph on a capture stream of the system's own, and replays it with one launch per
 * trial instead of about thirty.  The kernels and their arguments are the same, so the
 * results are bitwise those of the eager run.  Replay needs the KS_HARTREE_PCG_FD solver
 * (or no Hartree term) and timers off; otherwise the run is eager.  The instantiated
 * graphs live for one ks_minimize call.  In ks_minimize_batch, when every member has
 * graphs on, a lockstep tick whose members all have their factor queued is captured once
 * per ordered membership and replayed (the launches read each member's current slot from
 * device memory), again bitwise equal to the eager tick.  Errors: KS_E_INVAL, KS_E_HIP. */
int ks_enable_graphs(ks_system* s, int on);

/* ---- instrumentation ------------------------------------------------------------------ */

/* Turns the phase timers on (on != 0) or off.  While on, the library records a pair of
 * HIP events on the system's stream around every phase of the timeline above and
 * accumulates their elapsed times at the next synchronisation point.  Off by default;
 * the timers add two event records per phase. */
int ks_enable_timers(ks_system* s, int on);

/* Restricts the timers to the phases whose bit (1u << KS_PH_*) is set in mask, so that a
 * measurement of one kernel costs two event records per launch of that kernel only.
 * ks_enable_timers resets the mask to all phases.  Errors: KS_E_INVAL. */
int ks_timer_phases(ks_system* s, unsigned mask);

/* Copies the accumulated phase times into *out (host); reset != 0 clears them. */
int ks_read_timers(ks_system* s, ks_phase_times* out, int reset);

#ifdef __cplusplus
}
#endif
#endif /* KS_H */
