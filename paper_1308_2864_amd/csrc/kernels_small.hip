// Small dense FP64 algebra of the Stiefel step and the scalar logic of Alg. 3.
//
// One workgroup per system works on p x p (QR) or 2p x 2p (WY) matrices held in LDS
// when they fit, otherwise in a global scratch area of the workspace:
//  * Cholesky QR factor (Alg. 2 applied to Y = X - tau grad E): Y^T Y is assembled from
//    the Gram blocks of [X, D] as X^T X - tau (X^T D + D^T X) + tau^2 D^T D, factored as
//    R^T R, and the retraction weights A = R^{-1}, B = -tau R^{-1} give
//    X+ = X A + D B = Y R^{-1} (eq. (QR)).
//  * Cayley/SMW factor (eq. (WY3)): I + tau/2 V^T U with U = [G, X], V = [X, -G] is
//    assembled from the Gram blocks of [X, G], solved against V^T X by LU with partial
//    pivoting, giving X+ = X (I - tau Z_2) + G (-tau Z_1).  When X+^T X+ (computed from
//    the same Gram blocks) drifts from I by more than the re-orthonormalisation
//    threshold (Section 4.1), the Cholesky QR of X+ is folded into the weights.
//  * Barzilai-Borwein step (eq. (bb-1)), nonmonotone Armijo test and reference-value
//    update (eq. (NMLS-Armijo)), stopping rules of Section 4.1.
#include <mutex>
#include <vector>
#include <algorithm>
#include "ks_common.h"
#include "../../include/ks.h"

namespace ks {

namespace {

// ---- block-cooperative helpers (all threads of the block call them) -----------------

// A pivot is taken as a breakdown when it is not positive, not finite, or below
// kPivotTol times the original diagonal entry: the matrix is then singular to working
// precision (its condition number exceeds ~1/kPivotTol) and R^{-1} would be meaningless.
constexpr double kPivotTol = 1e-13;

// In-place upper Cholesky: on return M[i][j], j >= i, holds R with R^T R = M (input);
// the strict lower part is zeroed.  Returns nonzero on a breakdown pivot (see kPivotTol).
__device__ int blk_cholesky_upper(double* M, int ld, int p) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < p; ++k) {
    if (threadIdx.x == 0) {
      const double d = M[k * ld + k];
      // the original diagonal entry is the pivot plus the squares above it in column k
      double d0 = d;
      for (int m = 0; m < k; ++m) d0 += M[m * ld + k] * M[m * ld + k];
      if (!(d > kPivotTol * d0) || !isfinite(d)) bad = 1;
      else M[k * ld + k] = sqrt(d);
    }
    __syncthreads();
    if (bad) return 1;
    const double rkk = M[k * ld + k];
    for (int j = k + 1 + threadIdx.x; j < p; j += blockDim.x) M[k * ld + j] /= rkk;
    __syncthreads();
    const int m = p - k - 1;
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
      const int i = k + 1 + e / m, j = k + 1 + e % m;
      if (j >= i) M[i * ld + j] -= M[k * ld + i] * M[k * ld + j];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    if (i > j) M[i * ld + j] = 0.0;
  }
  __syncthreads();
  return 0;
}

// W = R^{-1} for upper triangular R (back substitution, one column per thread).
__device__ void blk_upper_inverse(const double* R, int ldr, double* W, int ldw, int p) {
  for (int j = threadIdx.x; j < p; j += blockDim.x) {
    for (int i = p - 1; i > j; --i) W[i * ldw + j] = 0.0;
    W[j * ldw + j] = 1.0 / R[j * ldr + j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int k = i + 1; k <= j; ++k) s += R[i * ldr + k] * W[k * ldw + j];
      W[i * ldw + j] = -s / R[i * ldr + i];
    }
  }
  __syncthreads();
}

// C = op(A) op(B) (p x p), op = transpose if the flag is set.  C must not alias A or B.
__device__ void blk_gemm(double* C, int ldc, const double* A, int lda, bool ta, const double* B,
                         int ldb, bool tb, int p) {
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    double s = 0.0;
    for (int k = 0; k < p; ++k) {
      const double a = ta ? A[k * lda + i] : A[i * lda + k];
      const double b = tb ? B[j * ldb + k] : B[k * ldb + j];
      s += a * b;
    }
    C[i * ldc + j] = s;
  }
  __syncthreads();
}

// Solves S Z = RHS in place (S: m x m, RHS: m x nr -> Z) by LU with partial pivoting
// (largest |pivot|, first index on ties).  Returns nonzero if a pivot is exactly zero or
// not finite.
__device__ int blk_lu_solve(double* S, int lds, int m, double* RHS, int ldb, int nr) {
  __shared__ double bv[kBlock];
  __shared__ int bi[kBlock];
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < m; ++k) {
    // pivot search
    double best = -1.0;
    int besti = m;
    for (int i = k + threadIdx.x; i < m; i += blockDim.x) {
      const double v = fabs(S[i * lds + k]);
      if (v > best) { best = v; besti = i; }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = besti;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) {
        const double v2 = bv[threadIdx.x + o];
        const int i2 = bi[threadIdx.x + o];
        if (v2 > bv[threadIdx.x] || (v2 == bv[threadIdx.x] && i2 < bi[threadIdx.x])) {
          bv[threadIdx.x] = v2;
          bi[threadIdx.x] = i2;
        }
      }
      __syncthreads();
    }
    const int piv = bi[0];
    if (threadIdx.x == 0 && (!(bv[0] > 0.0) || !isfinite(bv[0]))) bad = 1;
    __syncthreads();
    if (bad) return 1;
    if (piv != k) {
      for (int j = threadIdx.x; j < m; j += blockDim.x) {
        const double t = S[k * lds + j];
        S[k * lds + j] = S[piv * lds + j];
        S[piv * lds + j] = t;
      }
      for (int j = threadIdx.x; j < nr; j += blockDim.x) {
        const double t = RHS[k * ldb + j];
        RHS[k * ldb + j] = RHS[piv * ldb + j];
        RHS[piv * ldb + j] = t;
      }
    }
    __syncthreads();
    const double skk = S[k * lds + k];
    for (int i = k + 1 + threadIdx.x; i < m; i += blockDim.x) S[i * lds + k] /= skk;
    __syncthreads();
    const int rem = m - k - 1;
    for (int e = threadIdx.x; e < rem * rem; e += blockDim.x) {
      const int i = k + 1 + e / rem, j = k + 1 + e % rem;
      S[i * lds + j] -= S[i * lds + k] * S[k * lds + j];
    }
    for (int e = threadIdx.x; e < rem * nr; e += blockDim.x) {
      const int i = k + 1 + e / nr, j = e % nr;
      RHS[i * ldb + j] -= S[i * lds + k] * RHS[k * ldb + j];
    }
    __syncthreads();
  }
  // back substitution with the upper factor, one right-hand side per thread
  for (int c = threadIdx.x; c < nr; c += blockDim.x) {
    for (int i = m - 1; i >= 0; --i) {
      double s = RHS[i * ldb + c];
      for (int j = i + 1; j < m; ++j) s -= S[i * lds + j] * RHS[j * ldb + c];
      RHS[i * ldb + c] = s / S[i * lds + i];
    }
  }
  __syncthreads();
  return 0;
}

__device__ void blk_store_padded(double* dst, int pp, const double* src, int lds, int p,
                                 double scale) {
  for (int e = threadIdx.x; e < pp * pp; e += blockDim.x) {
    const int i = e / pp, j = e % pp;
    dst[e] = (i < p && j < p) ? scale * src[i * lds + j] : 0.0;
  }
  __syncthreads();
}

__device__ inline double* work_base(double* glob) {
  extern __shared__ double dyn[];
  return glob ? glob : dyn;
}

// ---- QR retraction weights -----------------------------------------------------------
// xx: X^T X; gxd: [., X^T D, D^T D] (pp x pp blocks).

// Wide blocks (p > 64): a right-looking Cholesky of M = Y^T Y whose pivots are judged
// against the saved diagonal, then R^{-1} in place: for k = p-1 .. 0, row k (already
// reduced by the rows below it) is scaled by 1/R_kk and eliminated from the rows above,
// whose column k still holds R and is read first.  Every step is one parallel update of
// the block (1024 threads); M sits in LDS up to p = 128 and in the scratch area above.
constexpr int kQrWideThreads = 1024;
constexpr int kQrWideMaxP = 512;
constexpr size_t kQrWideStatic = 3 * kQrWideMaxP * sizeof(double) + 1024;

__global__ __launch_bounds__(kQrWideThreads) void k_qr_factor_wide(
    const double* __restrict__ xx, const double* __restrict__ gxd, int p, int pp,
    const double* __restrict__ tau_p, double* __restrict__ A, double* __restrict__ B,
    double* glob, int* status) {
  __shared__ double d0[kQrWideMaxP], rk[kQrWideMaxP], ck[kQrWideMaxP];
  __shared__ int bad;
  double* M = work_base(glob);
  const int t = threadIdx.x, nt = blockDim.x;
  const int lane = t % kWave, wv = t / kWave, nw = nt / kWave;
  const double tau = *tau_p;
  const double* XD = gxd + (size_t)pp * pp;
  const double* DD = gxd + 2 * (size_t)pp * pp;
  for (int e = t; e < p * p; e += nt) {
    const int i = e / p, j = e % p;
    M[e] = xx[i * pp + j] - tau * (XD[i * pp + j] + XD[j * pp + i]) + tau * tau * DD[i * pp + j];
  }
  if (t == 0) bad = 0;
  __syncthreads();
  for (int i = t; i < p; i += nt) d0[i] = M[i * p + i];
  __syncthreads();
  for (int k = 0; k < p; ++k) {
    if (t == 0) {
      const double d = M[k * p + k];
      if (!(d > kPivotTol * d0[k]) || !isfinite(d)) bad = 1;
      else M[k * p + k] = sqrt(d);
    }
    __syncthreads();
    if (bad) {
      if (t == 0) *status = KS_E_NOT_SPD;
      return;
    }
    const double rkk = M[k * p + k];
    for (int j = k + 1 + t; j < p; j += nt) {
      const double v = M[k * p + j] / rkk;
      M[k * p + j] = v;
      rk[j] = v;
    }
    __syncthreads();
    // upper triangle of the trailing block: a wavefront per row, lanes along the row
    for (int i = k + 1 + wv; i < p; i += nw) {
      const double ri = rk[i];
      for (int j = i + lane; j < p; j += kWave) M[i * p + j] -= ri * rk[j];
    }
    __syncthreads();
  }
  for (int k = p - 1; k >= 0; --k) {
    const double inv = 1.0 / M[k * p + k];
    for (int j = k + t; j < p; j += nt) {
      const double w = j == k ? inv : M[k * p + j] * inv;
      rk[j] = w;
      M[k * p + j] = w;
    }
    for (int i = t; i < k; i += nt) ck[i] = M[i * p + k];
    __syncthreads();
    for (int i = wv; i < k; i += nw) {
      const double ci = ck[i];
      for (int j = k + lane; j < p; j += kWave)
        M[i * p + j] = (j == k ? 0.0 : M[i * p + j]) - ci * rk[j];
    }
    __syncthreads();
  }
  for (int e = t; e < pp * pp; e += nt) {
    const int i = e / pp, j = e % pp;
    const double w = (i < p && j < p && j >= i) ? M[i * p + j] : 0.0;
    A[e] = w;
    B[e] = -tau * w;
  }
}

// Blocked form for p > 128 (the matrix in global memory): 64-column blocks; one workgroup
// factors and inverts each diagonal block in LDS (pivots judged against the saved
// diagonal, as above), the panel R_KJ = R_KK^-T M_KJ and the trailing update
// M_IJ -= R_KI^T R_KJ are multi-workgroup products, and W = R^-1 follows by row blocks from
// the bottom, W_I = R_II^-1 (E_I - sum_{K > I} R_IK W_K).  A breakdown sets a flag that
// every later step reads, and A, B are then left untouched.
constexpr int kWB = 64;

__global__ void k_wf_assemble(const double* __restrict__ xx, const double* __restrict__ gxd,
                              int p, int pp, const double* __restrict__ tau_p,
                              double* __restrict__ M, double* __restrict__ R,
                              double* __restrict__ d0, double* __restrict__ flag) {
  const double tau = *tau_p;
  const double* XD = gxd + (size_t)pp * pp;
  const double* DD = gxd + 2 * (size_t)pp * pp;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < (size_t)p * p;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / p), j = (int)(e % p);
    const double v =
        xx[i * pp + j] - tau * (XD[i * pp + j] + XD[j * pp + i]) + tau * tau * DD[i * pp + j];
    M[e] = v;
    R[e] = 0.0;
    if (i == j) d0[i] = v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 0.0;
}

// Cholesky and inverse of diagonal block K (b = min(64, p - 64 K) columns) in LDS.
__global__ __launch_bounds__(1024) void k_wf_diag(const double* __restrict__ M, int p, int K,
                                                  const double* __restrict__ d0,
                                                  double* __restrict__ R, double* __restrict__ Ri,
                                                  double* __restrict__ flag, int* status) {
  __shared__ double S[kWB][kWB + 1];
  __shared__ double rk[kWB], ck[kWB];
  __shared__ int bad;
  if (*flag != 0.0) return;
  const int t = threadIdx.x, nt = blockDim.x;
  const int lane = t % kWave, wv = t / kWave, nw = nt / kWave;
  const int k0 = K * kWB, b = min(kWB, p - k0);
  for (int e = t; e < kWB * kWB; e += nt) {
    const int i = e / kWB, j = e % kWB;
    S[i][j] = (i < b && j < b) ? M[(size_t)(k0 + i) * p + k0 + j] : 0.0;
  }
  if (t == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < b; ++k) {
    if (t == 0) {
      const double d = S[k][k];
      if (!(d > kPivotTol * d0[k0 + k]) || !isfinite(d)) bad = 1;
      else S[k][k] = sqrt(d);
    }
    __syncthreads();
    if (bad) {
      if (t == 0) {
        *flag = 1.0;
        *status = KS_E_NOT_SPD;
      }
      return;
    }
    const double rkk = S[k][k];
    for (int j = k + 1 + t; j < b; j += nt) {
      const double v = S[k][j] / rkk;
      S[k][j] = v;
      rk[j] = v;
    }
    __syncthreads();
    for (int i = k + 1 + wv; i < b; i += nw) {
      const double ri = rk[i];
      for (int j = i + lane; j < b; j += kWave) S[i][j] -= ri * rk[j];
    }
    __syncthreads();
  }
  // R_KK (upper, zero below) into R
  for (int e = t; e < b * b; e += nt) {
    const int i = e / b, j = e % b;
    R[(size_t)(k0 + i) * p + k0 + j] = j >= i ? S[i][j] : 0.0;
  }
  __syncthreads();
  // R_KK^-1 in place (right-looking elimination from the last row)
  for (int k = b - 1; k >= 0; --k) {
    const double inv = 1.0 / S[k][k];
    for (int j = k + t; j < b; j += nt) {
      const double w = j == k ? inv : S[k][j] * inv;
      rk[j] = w;
      S[k][j] = w;
    }
    for (int i = t; i < k; i += nt) ck[i] = S[i][k];
    __syncthreads();
    for (int i = wv; i < k; i += nw) {
      const double ci = ck[i];
      for (int j = k + lane; j < b; j += kWave) S[i][j] = (j == k ? 0.0 : S[i][j]) - ci * rk[j];
    }
    __syncthreads();
  }
  for (int e = t; e < kWB * kWB; e += nt) {
    const int i = e / kWB, j = e % kWB;
    Ri[e] = (i < b && j < b && j >= i) ? S[i][j] : 0.0;
  }
}

// C (m x n, ldc) = beta C + alpha op(A) B with op(A)[i][k] = A[k][i] (transA) or A[i][k];
// 16 x 16 output tiles, 16-wide contraction slices through LDS.  Nothing when *flag is set.
struct WfGemm {
  const double* A;
  int lda;
  int transA;
  const double* B;
  int ldb;
  double* C;
  int ldc;
  int m, n, k;
  double alpha, beta;
  const double* flag;
};

__global__ __launch_bounds__(256) void k_wf_gemm(WfGemm g) {
  __shared__ double As[16][17], Bs[16][17];
  if (*g.flag != 0.0) return;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
  const int ia = blockIdx.y * 16 + tx;  // row of op(A) this thread stages (transposed load)
  double acc = 0.0;
  for (int k0 = 0; k0 < g.k; k0 += 16) {
    if (g.transA) {
      // op(A)[ia][k0 + ty] = A[k0 + ty][ia]: lanes along ia read contiguous memory
      As[tx][ty] = (ia < g.m && k0 + ty < g.k) ? g.A[(size_t)(k0 + ty) * g.lda + ia] : 0.0;
    } else {
      As[ty][tx] = (i < g.m && k0 + tx < g.k) ? g.A[(size_t)i * g.lda + k0 + tx] : 0.0;
    }
    Bs[ty][tx] = (k0 + ty < g.k && j < g.n) ? g.B[(size_t)(k0 + ty) * g.ldb + j] : 0.0;
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) acc += As[ty][kk] * Bs[kk][tx];
    __syncthreads();
  }
  if (i < g.m && j < g.n) {
    double* c = g.C + (size_t)i * g.ldc + j;
    *c = (g.beta == 0.0 ? 0.0 : g.beta * *c) + g.alpha * acc;
  }
}

// Rows 64 I .. of the identity (b x p): the right-hand side of a row block of R W = I.
__global__ void k_wf_eye(double* __restrict__ T, int b, int p, int I,
                         const double* __restrict__ flag) {
  if (*flag != 0.0) return;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < (size_t)b * p;
       e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / p), c = (int)(e % p);
    T[e] = c == kWB * I + r ? 1.0 : 0.0;
  }
}

__global__ void k_wf_store(const double* __restrict__ W, int p, int pp,
                           const double* __restrict__ tau_p, double* __restrict__ A,
                           double* __restrict__ B, const double* __restrict__ flag) {
  if (*flag != 0.0) return;
  const double tau = *tau_p;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < (size_t)pp * pp;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / pp), j = (int)(e % pp);
    const double w = (i < p && j < p && j >= i) ? W[(size_t)i * p + j] : 0.0;
    A[e] = w;
    B[e] = -tau * w;
  }
}

void wf_gemm(const WfGemm& g, hipStream_t st) {
  if (g.m <= 0 || g.n <= 0) return;
  hipLaunchKernelGGL(k_wf_gemm, dim3((g.n + 15) / 16, (g.m + 15) / 16), dim3(256), 0, st, g);
}

// The blocked factor; work holds 3 p^2 + 129 p + 4096 doubles (within small_work_doubles).
void launch_qr_factor_blocked(const double* xx, const double* gxd, int p, int pp,
                              const double* tau, double* A, double* B, double* work,
                              int* status, hipStream_t st) {
  const int nb = (p + kWB - 1) / kWB;
  const size_t p2 = (size_t)p * p;
  double* M = work;
  double* R = M + p2;
  double* W = R + p2;
  double* T = W + p2;                       // kWB x p
  double* Ri = T + (size_t)kWB * p;         // nb blocks of kWB x kWB
  double* d0 = Ri + (size_t)nb * kWB * kWB; // p
  double* flag = d0 + p;
  const int eb = (int)std::min<size_t>((p2 + 255) / 256, 4096);
  hipLaunchKernelGGL(k_wf_assemble, dim3(eb), dim3(256), 0, st, xx, gxd, p, pp, tau, M, R, d0,
                     flag);
  for (int K = 0; K < nb; ++K) {
    const int k0 = K * kWB, b = std::min(kWB, p - k0), r0 = k0 + b, rest = p - r0;
    double* RiK = Ri + (size_t)K * kWB * kWB;
    hipLaunchKernelGGL(k_wf_diag, dim3(1), dim3(1024), 0, st, M, p, K, d0, R, RiK, flag,
                       status);
    if (rest <= 0) continue;
    // panel: R[k0.., r0..] = R_KK^-T M[k0.., r0..]
    wf_gemm(WfGemm{RiK, kWB, 1, M + (size_t)k0 * p + r0, p, R + (size_t)k0 * p + r0, p, b, rest,
                   b, 1.0, 0.0, flag},
            st);
    // trailing: M[r0.., r0..] -= R[k0.., r0..]^T R[k0.., r0..]
    wf_gemm(WfGemm{R + (size_t)k0 * p + r0, p, 1, R + (size_t)k0 * p + r0, p,
                   M + (size_t)r0 * p + r0, p, rest, rest, b, -1.0, 1.0, flag},
            st);
  }
  for (int I = nb - 1; I >= 0; --I) {
    const int i0 = I * kWB, b = std::min(kWB, p - i0), r0 = i0 + b, rest = p - r0;
    const int tb = (int)std::min<size_t>(((size_t)b * p + 255) / 256, 4096);
    hipLaunchKernelGGL(k_wf_eye, dim3(tb), dim3(256), 0, st, T, b, p, I, flag);
    if (rest > 0)  // T -= R[i0.., r0..] W[r0.., :]
      wf_gemm(WfGemm{R + (size_t)i0 * p + r0, p, 0, W + (size_t)r0 * p, p, T, p, b, p, rest,
                     -1.0, 1.0, flag},
              st);
    // W[i0.., :] = R_II^-1 T
    wf_gemm(WfGemm{Ri + (size_t)I * kWB * kWB, kWB, 0, T, p, W + (size_t)i0 * p, p, b, p, b, 1.0,
                   0.0, flag},
            st);
  }
  const int sb = (int)std::min<size_t>(((size_t)pp * pp + 255) / 256, 4096);
  hipLaunchKernelGGL(k_wf_store, dim3(sb), dim3(256), 0, st, W, p, pp, tau, A, B, flag);
}

// Factor for p <= P (P = 16, 32, 64) by elimination on the augmented matrix [M | I]
// (M = Y^T Y padded to P x P with the identity, whose factor is the identity, so the padding
// leaves the p x p result unchanged and needs no guards).  Step k eliminates below the
// pivot with row k of the partly eliminated array: x[r][.] -= M'[k][r] x[k][.] / M'[k][k]
// for r > k (M'[r][k] = M'[k][r] by symmetry: the row operation of M = L D L^T).  After P
// steps the identity half holds L^{-1}; with R = D^{1/2} L^T (M = R^T R, R upper),
// R^{-1} = L^{-T} D^{-1/2}, so no back substitution is needed:
// W[i][j] = (L^{-1})[j][i] / sqrt(d_j).
// Only the upper triangle of M' and the strict lower triangle of L^{-1} (whose diagonal stays
// 1 and upper part 0) are ever needed, and together they fill one P x P square: element
// (r, c) is M'[r][c] for r <= c and L^{-1}[r][c] for r > c, kE elements per thread.  Row k
// of the square is then exactly the multiplier row of step k; its owners publish it (two
// buffers by step parity, so a step needs one barrier) and the owner of the pivot also
// publishes 1 / M'[k][k] and makes the pivot test.
template <int P>
constexpr int qr_factor_threads() {
  return P * P < 1024 ? P * P : 1024;
}

template <int P>
__device__ inline void k_qr_factor_aug_body(const QrFactor2dArgs& ka) {
  constexpr int kT = qr_factor_threads<P>();
  constexpr int kE = P * P / kT;
  const double* xx = ka.xx;
  const double* gxd = ka.gxd;
  if (ka.sel) {
    // launched ahead of the host's read of the line-search record: the same decisions the
    // host is about to take, from the same record
    const LsState* ls = ka.sel;
    if (ls->hartree_pending || ls->stop != KS_STOP_NONE || ls->error) return;
    if (!ls->accepted) {
      xx = ka.xx_rej;
      gxd = ka.gxd_rej;
    }
  }
  const int p = ka.p, pp = ka.pp;
  __shared__ double row[2][P];
  __shared__ double rinv[2];
  __shared__ double Ws[P][P + 1];
  __shared__ int bad;
  const int t = threadIdx.x;
  const double tau = *ka.tau_p;
  const double* XD = gxd + pp * pp;
  const double* DD = gxd + 2 * pp * pp;
  if (t == 0) bad = 0;
  // the pivot test of row r against the diagonal entry of M
  auto test = [&](double d, double d0) {
    if (!(d > kPivotTol * d0) || !isfinite(d)) bad = 1;
  };
  // M = X^T X - tau (X^T D + D^T X) + tau^2 D^T D (upper triangle); L^{-1} starts at 0
  double x[kE], d0[kE];
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int e = t + q * kT, r = e / P, c = e % P;
    const bool in = r < p && c < p;
    const int a = in ? r * pp + c : 0, b = in ? c * pp + r : 0;
    const double m = xx[a] - tau * (XD[a] + XD[b]) + tau * tau * DD[a];
    x[q] = r > c ? 0.0 : (in ? m : (r == c ? 1.0 : 0.0));
    d0[q] = x[q];
  }
  __syncthreads();  // bad = 0 before any test
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int e = t + q * kT, r = e / P, c = e % P;
    if (r == 0) {
      row[0][c] = x[q];
      if (c == 0) {
        rinv[0] = 1.0 / x[q];
        test(x[q], d0[q]);
      }
    }
  }
  __syncthreads();
  // kept a loop: unrolled, the body (run once per launch) would be bound by instruction fetch
#pragma unroll 1
  for (int k = 0; k < P - 1; ++k) {
    const double* rk = row[k & 1];
    double* rn = row[(k + 1) & 1];
    const double dinv = rinv[k & 1];
#pragma unroll
    for (int q = 0; q < kE; ++q) {
      const int e = t + q * kT, r = e / P, c = e % P;
      if (r > k) {
        // x[k][c]: M'[k][c] (c >= k), or L^{-1}[k][c]: published (c < k), 1 (c = k), 0
        const double v = rk[c];
        const double xk = (r <= c || c < k) ? v : (c == k ? 1.0 : 0.0);
        x[q] = fma(-rk[r] * dinv, xk, x[q]);
        if (r == k + 1) {
          rn[c] = x[q];
          if (c == r) {
            rinv[(k + 1) & 1] = 1.0 / x[q];
            test(x[q], d0[q]);
          }
        }
      }
    }
    __syncthreads();
  }
  if (bad) {
    if (t == 0) *ka.status = KS_E_NOT_SPD;
    return;
  }
  // W[c][r] = L^{-1}[r][c] / sqrt(d_r) for r > c and 1 / sqrt(d_r) on the diagonal; the
  // pivots d_r sit on the diagonal of the square (row[.] no longer needed: reuse for them)
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int e = t + q * kT, r = e / P, c = e % P;
    if (r == c) Ws[r][P] = 1.0 / sqrt(x[q]);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kE; ++q) {
    const int e = t + q * kT, r = e / P, c = e % P;
    const double sr = Ws[r][P];
    Ws[c][r] = r > c ? x[q] * sr : (r == c ? sr : 0.0);
    // R[r][c] = M'[r][c] / sqrt(d_r) on and above the diagonal
    if (ka.R && r < pp && c < pp) ka.R[r * pp + c] = (r <= c && r < p && c < p) ? x[q] * sr : 0.0;
  }
  __syncthreads();
  for (int e = t; e < pp * pp; e += kT) {
    const int i = e / pp, j = e % pp;
    const double v = (i < p && j < p) ? Ws[i][j] : 0.0;
    ka.A[e] = v;
    ka.B[e] = -tau * v;
  }
}

template <int P>
__global__ __launch_bounds__(qr_factor_threads<P>()) void k_qr_factor_aug(QrFactor2dArgs ka) {
  k_qr_factor_aug_body<P>(ka);
}

template <int P>
__global__ __launch_bounds__(qr_factor_threads<P>()) void k_qr_factor_aug_batch(
    BatchPtrs<QrFactor2dArgs> b) {
  k_qr_factor_aug_body<P>(batch_arg(b, blockIdx.x));
}


// ---- Cayley / SMW retraction weights -------------------------------------------------
// gram: [X^T X, X^T G, G^T G] (pp x pp each).
__global__ void k_wy_factor(const double* __restrict__ gram, int p, int pp,
                            const double* __restrict__ tau_p, double reorth_tol,
                            double* __restrict__ A, double* __restrict__ B, double* glob,
                            int* status, int* reorth_flag) {
  double* base = work_base(glob);
  const int m = 2 * p;
  double* S = base;             // m x m     (phase 1)
  double* Z = base + m * m;     // m x p     (kept)
  double* Aw = base;            // p x p     (phase 2 reuses S)
  double* Bw = Aw + p * p;
  double* T1 = Bw + p * p;
  double* T2 = T1 + p * p;
  const double tau = *tau_p;
  const double* XX = gram;
  const double* XG = gram + pp * pp;
  const double* GG = gram + 2 * pp * pp;
  const double ht = 0.5 * tau;
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int i = e / m, j = e % m;
    double v;
    if (i < p && j < p) v = ht * XG[i * pp + j];                 // X^T G
    else if (i < p) v = ht * XX[i * pp + (j - p)];                // X^T X
    else if (j < p) v = -ht * GG[(i - p) * pp + j];               // -G^T G
    else v = -ht * XG[(j - p) * pp + (i - p)];                    // -G^T X
    S[e] = v + (i == j ? 1.0 : 0.0);
  }
  for (int e = threadIdx.x; e < m * p; e += blockDim.x) {
    const int i = e / p, c = e % p;
    Z[e] = (i < p) ? XX[i * pp + c] : -XG[c * pp + (i - p)];   // V^T X = [X^T X; -G^T X]
  }
  __syncthreads();
  if (blk_lu_solve(S, m, m, Z, p, p)) {
    if (threadIdx.x == 0) *status = KS_E_SINGULAR;
    return;
  }
  // X+ = X (I - tau Z2) + G (-tau Z1)
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    Aw[e] = (i == j ? 1.0 : 0.0) - tau * Z[(p + i) * p + j];
    Bw[e] = -tau * Z[i * p + j];
  }
  __syncthreads();
  // X+^T X+ = A^T XX A + A^T XG B + (A^T XG B)^T + B^T GG B
  double* P = Z;  // Z no longer needed (m x p >= p x p)
  blk_gemm(T1, p, XX, pp, false, Aw, p, false, p);   // XX A
  blk_gemm(T2, p, Aw, p, true, T1, p, false, p);     // A^T XX A
  blk_gemm(T1, p, XG, pp, false, Bw, p, false, p);   // XG B
  blk_gemm(P, p, Aw, p, true, T1, p, false, p);      // A^T XG B
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    T2[e] += P[i * p + j] + P[j * p + i];
  }
  __syncthreads();
  blk_gemm(T1, p, GG, pp, false, Bw, p, false, p);   // GG B
  blk_gemm(P, p, Bw, p, true, T1, p, false, p);      // B^T GG B
  __shared__ double onrm;
  __shared__ double red[kBlock];
  double acc = 0.0;
  for (int e = threadIdx.x; e < p * p; e += blockDim.x) {
    const int i = e / p, j = e % p;
    const double v = T2[e] + P[e];
    T2[e] = v;
    const double dlt = v - (i == j ? 1.0 : 0.0);
    acc += dlt * dlt;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)blockDim.x; ++i) s += red[i];
    onrm = sqrt(s);
  }
  __syncthreads();
  if (onrm > reorth_tol) {
    // Cholesky QR of X+: fold R^{-1} into the weights
    if (blk_cholesky_upper(T2, p, p)) {
      if (threadIdx.x == 0) *status = KS_E_NOT_SPD;
      return;
    }
    blk_upper_inverse(T2, p, P, p, p);
    blk_gemm(T1, p, Aw, p, false, P, p, false, p);
    blk_store_padded(A, pp, T1, p, p, 1.0);
    blk_gemm(T1, p, Bw, p, false, P, p, false, p);
    blk_store_padded(B, pp, T1, p, p, 1.0);
    if (threadIdx.x == 0 && reorth_flag) *reorth_flag += 1;
  } else {
    blk_store_padded(A, pp, Aw, p, p, 1.0);
    blk_store_padded(B, pp, Bw, p, p, 1.0);
  }
}

// ---- gradient weights: W = -(X^T G)^T = -G^T X -------------------------------------
__global__ void k_grad_weights(const double* __restrict__ gram, int pp, double* __restrict__ W) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= pp * pp) return;
  const int i = e / pp, j = e % pp;
  W[e] = -gram[pp * pp + j * pp + i];
}

// ---- evaluation summary ----------------------------------------------------------------
__device__ void ls_judge(const EvalOut* ev, LsState* ls, LsState s, const LsParams& prm,
                         bool cg_pending);

// The evaluation summary: sums the per-block partials of every scalar slot (fixed
// order), forms the energy terms, ||X^T X - I||_F (or X^T B X) from the Gram block and,
// with ls, runs the line-search judgement on the result (one launch for all three).
constexpr int kFinishThreads = 1024;

__device__ inline void k_finish_eval_body(const FinishEvalArgs& ka, int ks_bid, int ks_nb) {
  const double* __restrict__ part = ka.part;
  int stride = ka.stride;
  ScalarCounts nb = ka.nb;
  double* __restrict__ sums = ka.sums;
  const double* __restrict__ xx = ka.xx;
  int p = ka.p;
  int pp = ka.pp;
  double f = ka.f;
  double dV = ka.dV;
  const double* enuc = ka.enuc;
  const CgState* cg = ka.cg;
  EvalOut* out = ka.out;
  LsState* ls = ka.ls;
  LsParams prm = ka.prm;
  (void)ks_bid;
  (void)ks_nb;

  __shared__ double sh[kFinishThreads / kWave];
  __shared__ double red[SL_COUNT];
  // the records thread 0 works on at the end, loaded now: their loads overlap the sums
  LsState s0{};
  double cg_rr = 0.0, cg_bb = 0.0, en = 0.0;
  int cg_it = 0, cg_done = 1;
  if (threadIdx.x == 0) {
    if (ls) s0 = *ls;
    if (cg) {
      cg_rr = cg->rr;
      cg_bb = cg->bb;
      cg_it = cg->it;
      cg_done = cg->done;
    }
    en = *enuc;
  }
  // one wavefront per value: slot w < SL_COUNT of the partials, then ||X^T X - I||_F^2 and
  // (bbr) sum_ij (I - R)_ij (X_t^T D_t)_ij; each lane sums its entries in order, then one
  // shuffle tree (a loop per wavefront keeps the code short: it runs once per launch and
  // would otherwise wait on instruction fetch)
  constexpr int kNW = kFinishThreads / kWave;
  static_assert(kNW >= SL_COUNT + 2, "one wavefront per value");
  __shared__ double wres[kNW];
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const bool bbr = ka.bbr_R != nullptr && ls != nullptr;
  double v = 0.0;
  if (wv < SL_COUNT) {
    int n = 0;
#pragma unroll
    for (int sl = 0; sl < SL_COUNT; ++sl)
      if (sl == wv) n = nb.v[sl];
    const double* __restrict__ q = part + (size_t)wv * stride;
#pragma unroll 8
    for (int i = lane; i < n; i += kWave) v += q[i];
  } else if (wv == SL_COUNT) {
    for (int e = lane; e < p * p; e += kWave) {
      const int i = e / p, j = e % p;
      const double d = xx[i * pp + j] - (i == j ? 1.0 : 0.0);
      v += d * d;
    }
  } else if (wv == SL_COUNT + 1 && bbr) {
    for (int e = lane; e < p * p; e += kWave) {
      const int i = e / p, j = e % p;
      v += ((i == j ? 1.0 : 0.0) - ka.bbr_R[i * pp + j]) * ka.bbr_xtd[i * pp + j];
    }
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
  if (lane == 0) wres[wv] = v;
  __syncthreads();
  (void)sh;
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int sl = 0; sl < SL_COUNT; ++sl) red[sl] = wres[sl];
  const double orth = wres[SL_COUNT], rxd = wres[SL_COUNT + 1];
  double acc = orth;
  for (int sl = 0; sl < SL_COUNT; ++sl) sums[sl] = red[sl];
  if (ka.cgw) {
    // the CG start of the Hartree solve whose residual the exchange pass measured (the
    // exact step counts as iteration 1)
    CgState* cs = ka.cgw;
    const double rr = red[SL_CGRR], bb = red[SL_CGBB];
    const double tol = ka.htol;
    cs->rr = rr;
    cs->bb = bb;
    cs->tol2 = tol * tol;
    cs->alpha = cs->beta = cs->pq = 0.0;
    cs->rz = 0.0;
    cs->rr_best = rr;
    cs->stall = 0;
    const int it = bb == 0.0 ? 0 : 1;
    const int done = (bb == 0.0 || !isfinite(rr) || !isfinite(bb) || rr <= tol * tol * bb) ? 1 : 0;
    cs->it = it;
    cs->maxit = ka.hmaxit;
    cs->done = done;
    if (cg == cs) {  // the record read below is the one just written
      cg_rr = rr;
      cg_bb = bb;
      cg_it = it;
      cg_done = done;
    }
  }
  EvalOut o;
  // the kinetic partial carries the weight mu; the Thomas-Fermi term is kinetic energy
  o.kinetic = 0.5 * f * red[SL_KIN] + dV * red[SL_TF];
  o.external = dV * red[SL_EXT];  // h^3 sum V_ext rho
  o.hartree = 0.5 * dV * red[SL_EH] + dV * red[SL_EBC] + (ka.ebc ? *ka.ebc : 0.0);
  o.xc = dV * red[SL_EX];
  o.nuclear = en;
  o.total = o.kinetic + o.external + o.hartree + o.xc + o.nuclear;
  o.g2 = red[SL_DD];
  if (bbr) {
    // QR trial X_t = (X_k - tau D_k) R^{-1}: with s = X_t - X_k = X_t (I - R) - tau D_k and
    // y = D_t - D_k, from ||s||^2 and <s, D_k> (retraction pass) and c = <D_k, D_t>
    // (gradient pass): <s, D_t> = sum (I - R) o (X_t^T D_t) - tau c,
    // ||y||^2 = ||D_t||^2 - 2 c + ||D_k||^2
    const double cr = red[SL_YY];
    o.ss = red[SL_SS];
    o.sy = rxd - s0.tau * cr - red[SL_SY];
    o.yy = red[SL_DD] - 2.0 * cr + s0.g2;
  } else {
    o.ss = red[SL_SS];
    o.sy = red[SL_SY];
    o.yy = red[SL_YY];
  }
  o.orth2 = acc;
  o.defect2 = red[SL_DEFECT];
  if (cg) {
    o.cg_iters = cg_it;
    o.cg_relres = cg_bb > 0.0 ? sqrt(cg_rr / cg_bb) : 0.0;
  } else {
    o.cg_iters = 0;
    o.cg_relres = 0.0;
  }
  o.nonfinite = (!isfinite(o.total) || !isfinite(o.g2)) ? 1 : 0;
  *out = o;
  if (ls) ls_judge(&o, ls, s0, prm, cg && !cg_done);
  if (ka.mirror) {
    // this thread's own writes above are the latest values of the records it copies
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2* src = static_cast<const d2*>(ka.mirror_src);
    d2* dst = static_cast<d2*>(ka.mirror);
    for (int i = 0; i < ka.mirror_bytes / 16; ++i) dst[i] = src[i];
  }
}

__global__ __launch_bounds__(1024) void k_finish_eval(FinishEvalArgs ka) {
  k_finish_eval_body(ka, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(1024) void k_finish_eval_batch(BatchPtrs<FinishEvalArgs> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_finish_eval_body(batch_arg(b, s), blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}


__global__ void k_set_scalar(double* d, double v) { *d = v; }

__global__ void k_ls_reset(LsState* ls) { *ls = LsState{}; }

// [3][pp][pp] padded Gram blocks -> [3][p][p]
__global__ void k_compact_gram(const double* __restrict__ g, int pp, int p,
                               double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * p * p) return;
  const int prod = e / (p * p), ij = e % (p * p), i = ij / p, j = ij % p;
  out[e] = g[(size_t)prod * pp * pp + i * pp + j];
}

// ---- Alg. 3 scalar logic -------------------------------------------------------------

__device__ double bb_tau(int k, double ss, double sy, double yy, const LsParams& prm) {
  if (k == 0) return prm.tau0;
  int rule = prm.bb_rule;
  if (rule == KS_BB_ALT) rule = (k % 2 == 1) ? KS_BB1 : KS_BB2;
  double t;
  if (rule == KS_BB1) t = (sy != 0.0) ? ss / fabs(sy) : INFINITY;
  else t = (yy != 0.0) ? fabs(sy) / yy : INFINITY;
  if (!isfinite(t) || !(t > 0.0)) t = prm.tau0;
  return fmin(fmax(t, prm.tau_min), prm.tau_max);
}

__global__ void k_ls_init(const EvalOut* ev, LsState* ls, LsParams prm) {
  LsState s = {};
  s.E = ev->total;
  s.g2 = ev->g2;
  s.C = s.E;
  s.Q = 1.0;
  s.k = 0;
  s.h = 0;
  s.tau_bb = bb_tau(0, 0.0, 0.0, 0.0, prm);
  s.tau = s.tau_bb;
  s.nfe = 1;
  s.accepted = 1;
  s.error = ls->error;  // a step before init may have flagged an error
  if (ev->nonfinite) {
    s.error = KS_E_NONFINITE;
    s.stop = KS_STOP_ERROR;
  } else if (s.E <= prm.energy_target) {
    s.stop = KS_STOP_ENERGY;
  } else if (sqrt(s.g2) <= prm.eps_g) {
    s.stop = KS_STOP_GRAD;
  } else if (prm.max_iter <= 0) {
    s.stop = KS_STOP_MAXIT;
  }
  if (s.error != 0) s.stop = KS_STOP_ERROR;
  *ls = s;
}

__global__ void k_ls_restart(const EvalOut* ev, LsState* ls, LsParams prm) {
  LsState s = *ls;
  s.nfe += 1;
  s.E = ev->total;
  s.g2 = ev->g2;
  s.C = s.E;
  s.Q = 1.0;
  s.h = 0;
  s.tau = s.tau_bb;
  s.accepted = 1;
  if (ev->nonfinite) {
    s.error = KS_E_NONFINITE;
    s.stop = KS_STOP_ERROR;
  } else if (s.stop == KS_STOP_NONE) {
    if (s.E <= prm.energy_target) s.stop = KS_STOP_ENERGY;
    else if (sqrt(s.g2) <= prm.eps_g) s.stop = KS_STOP_GRAD;
  }
  *ls = s;
}

// s: the record as read from ls at the start of the calling kernel.
__device__ void ls_judge(const EvalOut* ev, LsState* ls, LsState s, const LsParams& prm,
                         bool cg_pending) {
  if (cg_pending) {
    // the Hartree potential of this trial is not converged yet: the host finishes the
    // solve, re-evaluates the trial and judges it again
    s.hartree_pending = 1;
    *ls = s;
    return;
  }
  s.hartree_pending = 0;
  s.nfe += 1;
  if (ev->defect2 > kBf16Defect * kBf16Defect * ev->g2) s.bf16_off = 1;
  if (s.error != 0) {
    s.stop = KS_STOP_ERROR;
    *ls = s;
    return;
  }
  const double Et = ev->nonfinite ? INFINITY : ev->total;
  const double rhs = s.C - prm.rho1 * s.tau * s.g2;
  const bool ok = Et <= rhs;
  if (ok || s.h >= prm.h_max) {
    if (!isfinite(Et)) {
      s.error = KS_E_NONFINITE;
      s.stop = KS_STOP_ERROR;
      s.accepted = 0;
      *ls = s;
      return;
    }
    if (!ok) s.ls_fail += 1;
    s.accepted = 1;
    s.tau_acc = s.tau;
    const double df = fabs(s.E - Et) / (fabs(s.E) + 1.0);
    s.df[0] = s.df[1];
    s.df[1] = s.df[2];
    s.df[2] = df;
    s.ndf += 1;
    const double Qn = prm.eta * s.Q + 1.0;
    s.C = (prm.eta * s.Q * s.C + Et) / Qn;
    s.Q = Qn;
    s.E = Et;
    s.g2 = ev->g2;
    s.k += 1;
    if (Et <= prm.energy_target)
      s.stop = KS_STOP_ENERGY;
    else if (s.ndf >= 3 && (s.df[0] + s.df[1] + s.df[2]) / 3.0 < prm.stagnation_tol)
      s.stop = KS_STOP_STAGNATION;
    else if (sqrt(s.g2) <= prm.eps_g)
      s.stop = KS_STOP_GRAD;
    else if (s.k >= prm.max_iter)
      s.stop = KS_STOP_MAXIT;
    s.tau_bb = bb_tau(s.k, ev->ss, ev->sy, ev->yy, prm);
    s.h = 0;
    s.tau = s.tau_bb;
  } else {
    s.accepted = 0;
    s.h += 1;
    s.backtracks += 1;
    s.tau = s.tau_bb * pow(prm.delta, (double)s.h);
  }
  *ls = s;
}


size_t query_lds_limit() {
  int dev = 0, v = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    v = 65536;
  return (size_t)v;
}

size_t dyn_lds_limit() {
  static const size_t lim = query_lds_limit();  // initialised once, thread-safe
  return lim;
}

template <typename K>
bool prepare_lds(K kernel, size_t bytes) {
  // leave room for the kernel's static shared arrays
  // the limit set is the same for every size, so concurrent host threads agree on it
  if (bytes + 8192 > dyn_lds_limit()) return false;
  if (bytes > 32768)
    set_dyn_lds_once(reinterpret_cast<const void*>(kernel), (int)(dyn_lds_limit() - 8192));
  return true;
}

}  // namespace

size_t small_work_doubles(int p) {
  // WY: S (2p x 2p) and Z (2p x p), then four p x p matrices in place of S; QR: 2 p^2
  return (size_t)6 * p * p + 64;
}

void launch_ls_reset(LsState* ls, hipStream_t st) {
  hipLaunchKernelGGL(k_ls_reset, dim3(1), dim3(1), 0, st, ls);
}

void launch_compact_gram(const double* gram, int pp, int p, double* out, hipStream_t st) {
  const int total = 3 * p * p;
  hipLaunchKernelGGL(k_compact_gram, dim3((total + 255) / 256), dim3(256), 0, st, gram, pp, p,
                     out);
}

void launch_grad_weights(const double* gram, int pp, double* W, hipStream_t st) {
  hipLaunchKernelGGL(k_grad_weights, dim3((pp * pp + 255) / 256), dim3(256), 0, st, gram, pp, W);
}

void launch_qr_factor(const double* xx, const double* gxd, int p, int pp, const double* tau,
                      double* A, double* B, double* work, int* status, hipStream_t st,
                      double* R) {
  if (p <= 16) {
    hipLaunchKernelGGL(k_qr_factor_aug<16>, dim3(1), dim3(qr_factor_threads<16>()), 0, st,
                       QrFactor2dArgs{xx, gxd, p, pp, tau, A, B, status, nullptr, nullptr,
                                      nullptr, R});
    return;
  }
  if (p <= 32) {
    hipLaunchKernelGGL(k_qr_factor_aug<32>, dim3(1), dim3(qr_factor_threads<32>()), 0, st,
                       QrFactor2dArgs{xx, gxd, p, pp, tau, A, B, status, nullptr, nullptr,
                                      nullptr, R});
    return;
  }
  if (p <= 64) {
    hipLaunchKernelGGL(k_qr_factor_aug<64>, dim3(1), dim3(qr_factor_threads<64>()), 0, st,
                       QrFactor2dArgs{xx, gxd, p, pp, tau, A, B, status, nullptr, nullptr,
                                      nullptr, R});
    return;
  }
  if (p > 128) {
    launch_qr_factor_blocked(xx, gxd, p, pp, tau, A, B, work, status, st);
    return;
  }
  // M (p x p) in LDS when it fits beside the static arrays; the attribute value does not
  // depend on p, so concurrent host threads agree on it
  const size_t bytes = (size_t)p * p * sizeof(double);
  const bool lds = bytes + kQrWideStatic <= dyn_lds_limit();
  if (lds && bytes > 32768)
    set_dyn_lds_once(reinterpret_cast<const void*>(k_qr_factor_wide),
                     (int)(dyn_lds_limit() - kQrWideStatic));
  hipLaunchKernelGGL(k_qr_factor_wide, dim3(1), dim3(kQrWideThreads), lds ? bytes : 0, st, xx,
                     gxd, p, pp, tau, A, B, lds ? nullptr : work, status);
}

// C = A + B W for p x p blocks (stride pp; FP64): 16 x 16 output tiles, the contraction in
// 16-wide slices staged through LDS.  Used to form X^T D = X^T G + (X^T X) W (and
// X^T B D = X^T G + (X^T B X) W) from blocks already reduced, instead of a Gram pass over D.
__global__ __launch_bounds__(256) void k_small_gemm_add(const double* __restrict__ A,
                                                        const double* __restrict__ B,
                                                        const double* __restrict__ W,
                                                        double* __restrict__ C, int p, int pp) {
  __shared__ double Bs[16][17], Ws[16][17];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
  double acc = 0.0;
  for (int k0 = 0; k0 < p; k0 += 16) {
    Bs[ty][tx] = (i < p && k0 + tx < p) ? B[(size_t)i * pp + k0 + tx] : 0.0;
    Ws[ty][tx] = (k0 + ty < p && j < p) ? W[(size_t)(k0 + ty) * pp + j] : 0.0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += Bs[ty][k] * Ws[k][tx];
    __syncthreads();
  }
  if (i < p && j < p) C[(size_t)i * pp + j] = A[(size_t)i * pp + j] + acc;
}

void launch_small_gemm_add(const double* A, const double* B, const double* W, double* C, int p,
                           int pp, hipStream_t st) {
  const int t = (p + 15) / 16;
  hipLaunchKernelGGL(k_small_gemm_add, dim3(t, t), dim3(256), 0, st, A, B, W, C, p, pp);
}

// One 16 x 16 tile of (xx W) per block as in k_small_gemm_add, then the block's sum of
// (xg - xd + xx W)^2 over its tile, one partial per block in tile order.
__global__ __launch_bounds__(256) void k_bf16_defect(const double* __restrict__ xg,
                                                     const double* __restrict__ xd,
                                                     const double* __restrict__ xx,
                                                     const double* __restrict__ W, int p,
                                                     int pp, double* __restrict__ part) {
  __shared__ double Bs[16][17], Ws[16][17];
  __shared__ double sh[kBlock / kWave];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
  double acc = 0.0;
  for (int k0 = 0; k0 < p; k0 += 16) {
    Bs[ty][tx] = (i < p && k0 + tx < p) ? xx[(size_t)i * pp + k0 + tx] : 0.0;
    Ws[ty][tx] = (k0 + ty < p && j < p) ? W[(size_t)(k0 + ty) * pp + j] : 0.0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += Bs[ty][k] * Ws[k][tx];
    __syncthreads();
  }
  const double d =
      (i < p && j < p) ? xg[(size_t)i * pp + j] - xd[(size_t)i * pp + j] + acc : 0.0;
  const double s = block_sum(d * d, sh);
  if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = s;
}

int bf16_defect_blocks(int p) {
  const int t = (p + 15) / 16;
  return t * t;
}

void launch_bf16_defect(const double* xg, const double* xd, const double* xx, const double* W,
                        int p, int pp, double* part, hipStream_t st) {
  const int t = (p + 15) / 16;
  hipLaunchKernelGGL(k_bf16_defect, dim3(t, t), dim3(256), 0, st, xg, xd, xx, W, p, pp, part);
}

void launch_qr_factor_next(const QrFactor2dArgs& a, hipStream_t st) {
  if (a.p <= 16)
    hipLaunchKernelGGL(k_qr_factor_aug<16>, dim3(1), dim3(qr_factor_threads<16>()), 0, st, a);
  else if (a.p <= 32)
    hipLaunchKernelGGL(k_qr_factor_aug<32>, dim3(1), dim3(qr_factor_threads<32>()), 0, st, a);
  else
    hipLaunchKernelGGL(k_qr_factor_aug<64>, dim3(1), dim3(qr_factor_threads<64>()), 0, st, a);
}

// One column (the orbital-free problem): eq. (WY-1d) gives x+ = (1 - beta_2) x - beta_1 a
// with a = E_x in closed form from s = x^T x, t = a^T x, u = a^T a, two inner products
// instead of the 2 x 2 solve.  In the B metric the same scalars are x^T B x, x^T g and
// g^T B^{-1} g.  |x+|^2 drifting past reorth_tol rescales both weights.
__global__ void k_wy_factor_1d(const double* __restrict__ gram, int pp,
                               const double* __restrict__ tau_p, double reorth_tol,
                               double* __restrict__ A, double* __restrict__ B, int* status,
                               int* reorth_flag) {
  if (threadIdx.x != 0) return;
  const double tau = *tau_p, ht = 0.5 * tau;
  const double s = gram[0], t = gram[pp * pp], u = gram[2 * pp * pp];
  const double den = 1.0 - ht * ht * t * t + ht * ht * u * s;
  if (!(den != 0.0) || !isfinite(den)) {
    *status = KS_E_SINGULAR;
    return;
  }
  const double b1 = tau * s / den;
  const double b2 = -tau * (t + ht * (t * t - u * s)) / den;
  double a = 1.0 - b2, b = -b1;
  const double nrm2 = a * a * s + 2.0 * a * b * t + b * b * u;
  if (fabs(nrm2 - 1.0) > reorth_tol) {
    if (!(nrm2 > 0.0)) {
      *status = KS_E_NOT_SPD;
      return;
    }
    const double r = 1.0 / sqrt(nrm2);
    a *= r;
    b *= r;
    if (reorth_flag) *reorth_flag += 1;
  }
  for (int e = 0; e < pp * pp; ++e) {
    A[e] = e == 0 ? a : 0.0;
    B[e] = e == 0 ? b : 0.0;
  }
}

void launch_wy_factor(const double* gram_xg, int p, int pp, const double* tau,
                      double reorth_tol, double* A, double* B, double* work, int* status,
                      int* reorth_flag, hipStream_t st) {
  if (p == 1) {
    hipLaunchKernelGGL(k_wy_factor_1d, dim3(1), dim3(kWave), 0, st, gram_xg, pp, tau,
                       reorth_tol, A, B, status, reorth_flag);
    return;
  }
  const size_t bytes = small_work_doubles(p) * sizeof(double);
  const bool lds = prepare_lds(k_wy_factor, bytes);
  hipLaunchKernelGGL(k_wy_factor, dim3(1), dim3(kBlock), lds ? bytes : 0, st, gram_xg, p, pp,
                     tau, reorth_tol, A, B, lds ? nullptr : work, status, reorth_flag);
}

void launch_finish_eval(const double* part, int stride, const int* nblk, double* sums,
                        const double* gram_xx, int p, int pp, double f, double dV,
                        const double* enuc, const CgState* cg, EvalOut* out, LsState* ls,
                        const LsParams* prm, hipStream_t st, CgState* cgw, double htol,
                        int hmaxit, const double* ebc, const double* bbr_R,
                        const double* bbr_xtd, void* mirror, const void* mirror_src,
                        int mirror_bytes) {
  ScalarCounts nb{};
  for (int i = 0; i < SL_COUNT; ++i) nb.v[i] = nblk[i];
  hipLaunchKernelGGL(k_finish_eval, dim3(1), dim3(kFinishThreads), 0, st,
                     FinishEvalArgs{part, stride, nb, sums, gram_xx, p, pp, f, dV, enuc, cg, out,
                         ls, prm ? *prm : LsParams{}, cgw, htol, hmaxit, ebc, bbr_R,
                         bbr_xtd, mirror, mirror_src, mirror_bytes});
}

void launch_set_scalar(double* dst, double v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, st, dst, v);
}

void launch_ls_init(const EvalOut* ev, LsState* ls, LsParams prm, hipStream_t st) {
  hipLaunchKernelGGL(k_ls_init, dim3(1), dim3(1), 0, st, ev, ls, prm);
}

void launch_ls_restart(const EvalOut* ev, LsState* ls, LsParams prm, hipStream_t st) {
  hipLaunchKernelGGL(k_ls_restart, dim3(1), dim3(1), 0, st, ev, ls, prm);
}


// ---- batched launches ------------------------------------------------------------------

void launch_qr_factor_batch(const BatchPtrs<QrFactor2dArgs>& b, int p_max, hipStream_t st) {
  if (p_max <= 16)
    hipLaunchKernelGGL(k_qr_factor_aug_batch<16>, dim3(b.S), dim3(qr_factor_threads<16>()), 0, st, b);
  else if (p_max <= 32)
    hipLaunchKernelGGL(k_qr_factor_aug_batch<32>, dim3(b.S), dim3(qr_factor_threads<32>()), 0, st, b);
  else
    hipLaunchKernelGGL(k_qr_factor_aug_batch<64>, dim3(b.S), dim3(qr_factor_threads<64>()), 0, st, b);
}

void launch_finish_eval_batch(const BatchPtrs<FinishEvalArgs>& b, hipStream_t st) {
  hipLaunchKernelGGL(k_finish_eval_batch, dim3(b.S), dim3(kFinishThreads), 0, st, b);
}

namespace {
__global__ void k_gather(GatherArgs g) {
  const int s = blockIdx.x;
  const double* src = reinterpret_cast<const double*>(g.src[s]);
  double* dst = reinterpret_cast<double*>(g.dst + (size_t)s * g.bytes);
  for (int i = threadIdx.x; i < g.bytes / 8; i += blockDim.x) dst[i] = src[i];
}
}  // namespace

void launch_gather(const GatherArgs& g, hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3(g.S), dim3(64), 0, st, g);
}

namespace {
__global__ void k_set_ints(int* __restrict__ dst, IntList l) {
  if ((int)threadIdx.x < l.n) dst[threadIdx.x] = l.v[threadIdx.x];
}
}  // namespace

void launch_set_ints(int* dst, const IntList& l, hipStream_t st) {
  hipLaunchKernelGGL(k_set_ints, dim3(1), dim3(64), 0, st, dst, l);
}


void set_dyn_lds_once(const void* k, int bytes) {
  static std::mutex mu;
  static std::vector<const void*> done;
  std::lock_guard<std::mutex> lock(mu);
  if (std::find(done.begin(), done.end(), k) != done.end()) return;
  (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  done.push_back(k);
}

}  // namespace ks
