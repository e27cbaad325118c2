// Grid kernels of the energy/gradient assembly (the paper's "T0" part, Section 4.1):
// nuclear potential, density, Hartree conjugate gradients, Slater exchange and the
// 7-point Hamiltonian applied to the orbital block, with fused FP64 energy partials.
//
// Layout: n-vectors are double[n] in linear grid order g = i + nx*(j + ny*k); orbital
// blocks are n x ld row-major ("grid-major"): consecutive threads walk consecutive
// orbitals of one grid point, then the next point, so every wavefront load is one
// contiguous segment.
#include <cmath>

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

// E_II = sum over pairs a < b of Z_a Z_b / |R_a - R_b|: one block, thread t sums the rows
// a = t, t + blockDim, ... and the block adds the row sums in a fixed order.
__global__ void k_enuc(double* out, const double* R, const double* Z, int M) {
  __shared__ double sh[kBlock / kWave];
  double e = 0.0;
  for (int a = threadIdx.x; a < M; a += blockDim.x)
    for (int b = a + 1; b < M; ++b) {
      const double dx = R[3 * a] - R[3 * b], dy = R[3 * a + 1] - R[3 * b + 1],
                   dz = R[3 * a + 2] - R[3 * b + 2];
      e += Z[a] * Z[b] / sqrt(dx * dx + dy * dy + dz * dz);
    }
  e = block_sum(e, sh);
  if (threadIdx.x == 0) *out = e;
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

// ---- LDA correlation: Perdew and Zunger (1981), unpolarised ------------------------------
// Their parametrisation of the Ceperley-Alder electron-gas correlation energy per
// electron as a function of r_s = (3/(4 pi rho))^{1/3}, and v_c = d(rho eps_c)/d rho =
// eps_c - (r_s/3) d eps_c/d r_s written out per branch.
constexpr double kPzGamma = -0.1423, kPzBeta1 = 1.0529, kPzBeta2 = 0.3334;
constexpr double kPzA = 0.0311, kPzB = -0.048, kPzC = 0.0020, kPzD = -0.0116;

__device__ inline void pz81(double rho, double* ec, double* vc) {
  if (!(rho > 0.0)) {
    *ec = 0.0;
    *vc = 0.0;
    return;
  }
  const double rs = cbrt(3.0 / (4.0 * kPi * rho));
  if (rs >= 1.0) {
    const double sq = sqrt(rs);
    const double den = 1.0 + kPzBeta1 * sq + kPzBeta2 * rs;
    *ec = kPzGamma / den;
    *vc = kPzGamma * (1.0 + (7.0 / 6.0) * kPzBeta1 * sq + (4.0 / 3.0) * kPzBeta2 * rs) /
          (den * den);
  } else {
    const double l = log(rs);
    *ec = kPzA * l + kPzB + kPzC * rs * l + kPzD * rs;
    *vc = kPzA * l + (kPzB - kPzA / 3.0) + (2.0 / 3.0) * kPzC * rs * l +
          (2.0 * kPzD - kPzC) / 3.0 * rs;
  }
}

// Thomas-Fermi constant of Section 2.2 eq. (TFW): (3/10)(3 pi^2)^{2/3}
constexpr double kCtf = 2.871234000188191;

// ---- Slater exchange, effective potential, Hartree/exchange/external energy partials ---
// The external energy h^3 sum V_ext rho is summed here, from the density of the evaluated
// block (formed from its stored values), rather than as sum V_ext X^2 in the Hamiltonian
// pass: the same number up to summation order, without a V_ext stream in the stencil.

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
  double eh = 0.0, ex = 0.0, ee = 0.0, et = 0.0, rr = 0.0, bb = 0.0, eb = 0.0;
  const bool cg_check = ka.cg_check != 0;
  for (size_t g = beg + threadIdx.x; g < end; g += blockDim.x) {
    if (cg_check) {
      // the residual test of the Hartree solve, as the CG start forms it
      const int gi = (int)g;
      const int i = gi % gr.nx, j = (gi / gr.nx) % gr.ny, k = gi / (gr.nx * gr.ny);
      const double b = poisson_rhs(rho, gi, gr);
      const double ri = b - op_apply(vh, nullptr, 0.0, gi, i, j, k, gr);
      rr += ri * ri;
      bb += b * b;
    }
    const double r = rho[g];
    const double ve = vext[g];
    const double h = (use_h && !trivial) ? vh[g] : 0.0;
    double vx = 0.0, e = 0.0;
    if (use_x & 1) {  // Slater exchange
      const double c = cbrt(r);
      vx = -cv * c;
      e = -cx * c;
    }
    if (use_x & 2) {  // LDA correlation
      double ec, vc;
      pz81(r, &ec, &vc);
      vx += vc;
      e += ec;
    }
    if (use_x & 4) {  // Thomas-Fermi kinetic energy C_TF rho^{5/3}: kinetic, not xc
      const double c = cbrt(r), c2 = c * c;
      vx += (5.0 / 3.0) * kCtf * c2;
      et += r * kCtf * c2;
    }
    double vb = 0.0;
    if (ka.vbc) {
      vb = ka.vbc[g];
      eb += r * vb;
    }
    veff[g] = ve + h + vb + vx;
    eh += r * h;
    ex += r * e;
    ee += r * ve;
  }
  // the seven block sums: the values go through LDS and wavefront w sums values w and
  // w + 4 (each lane over four threads in thread order, then one shuffle tree), so the
  // code holds one tree instead of seven (it runs once per launch: instruction fetch)
  constexpr int kNV = 7;
  __shared__ double tv[kNV][kBlock];
  tv[0][threadIdx.x] = eh;
  tv[1][threadIdx.x] = ex;
  tv[2][threadIdx.x] = ee;
  tv[3][threadIdx.x] = et;
  tv[4][threadIdx.x] = eb;
  tv[5][threadIdx.x] = rr;
  tv[6][threadIdx.x] = bb;
  __syncthreads();
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  constexpr int kSlots[kNV] = {SL_EH, SL_EX, SL_EXT, SL_TF, SL_EBC, SL_CGRR, SL_CGBB};
#pragma unroll 1
  for (int k = w; k < kNV; k += kBlock / kWave) {
    double v = 0.0;
#pragma unroll
    for (int i = lane; i < kBlock; i += kWave) v += tv[k][i];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
    const bool wanted = k < 4 || (k == 4 && ka.vbc) || (k > 4 && cg_check);
    if (lane == 0 && wanted) pt.buf[(size_t)kSlots[k] * pt.stride + lb] = v;
  }
  (void)sh;
}

__global__ void k_xc(XcArgs ka) {
  k_xc_body(ka, blockIdx.x, gridDim.x);
}

__global__ void k_xc_batch(BatchPtrs<XcArgs> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_xc_body(batch_arg(b, s), blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}


// ---- Hamiltonian on the orbital block -----------------------------------------------
// Y = scale * ((1/2) L X + Diag(veff) X), L = -Laplacian_h (7 points, zero Dirichlet).
// With pt: per-block partials of sum X.(LX) (kinetic energy).

// A lane owns kW orbitals (a column pair when p, ld are even and the blocks are
// pair-aligned) of one grid column; consecutive lanes take consecutive orbitals of one
// point, then the next point, so a wavefront covers 64 consecutive (point, orbital group)
// entries of a plane and each of its loads is one contiguous segment.  A work item is such
// a wavefront slice over a run of kRun planes (16, or 8 when runs of 16 would leave
// wavefronts without an item), marched as in the Gram-fused form below: a software
// pipeline kHxPlainDepth planes deep issues the loads of plane k + kHxPlainDepth (centre
// one plane further, the four in-plane neighbours, V_eff) while plane k is computed, the
// z neighbours come from registers, and the run is unrolled completely.  All loads are
// branch-free (clamped addresses, zero outside the grid).
constexpr int kHxChunk = 8;
constexpr int kHxPlainDepth = 4;

template <typename T, int kW>
struct HxVec {
  typedef T type __attribute__((ext_vector_type(kW)));
};
template <typename T>
struct HxVec<T, 1> {
  typedef T type;
};

template <typename T, int kW>
__device__ inline double hx_elem(const typename HxVec<T, kW>::type& v, int e) {
  if constexpr (kW == 1) {
    (void)e;
    return (double)v;
  } else {
    return (double)v[e];
  }
}

template <typename T, bool kEnergy, int kW, int kRun>
__device__ inline void hx_items_run(const HxArgs<T>& ka, int lb, int nblk, double& kin) {
  typedef typename HxVec<T, kW>::type V;
  const T* __restrict__ X = ka.X;
  T* __restrict__ Y = ka.Y;
  const int ldx = ka.ldx, ldy = ka.ldy;
  const double* __restrict__ veff = ka.veff;
  const Grid gr = ka.gr;
  const int nx = gr.nx, ny = gr.ny, nz = gr.nz, nxy = nx * ny;
  const int pw = ka.p / kW;
  const int cols = nxy * pw;  // (point, orbital group) entries per plane
  const int groups = (cols + kWave - 1) / kWave;
  const int items = groups * ((nz + kRun - 1) / kRun);
  // element offsets fit 31 bits (n * ld < 2^31 is checked at system creation)
  const int sy = nx * ldx, szx = nxy * ldx, szy = nxy * ldy;
  const double ih2 = gr.inv_h2 * gr.mu, scale = ka.scale;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int nwaves = nblk * (kBlock / kWave);
  struct Stage {
    V zn, xm, xp, ym, yp;
    double ve;
  };
  for (int it = lb * (kBlock / kWave) + w; it < items; it += nwaves) {
    const int zc = it / groups, grp = it - zc * groups;
    const int t = grp * kWave + lane;
    const bool live = t < cols;
    const int tc = live ? t : 0;
    const int col = tc / pw, c = (tc - col * pw) * kW;
    const int i = col % nx, j = col / nx;
    const int k0 = zc * kRun, k1 = min(k0 + kRun, nz);
    const int o0 = col * ldx + c, oy = col * ldy + c;
    const bool hxm = live && i > 0, hxp = live && i < nx - 1;
    const bool hym = live && j > 0, hyp = live && j < ny - 1;
    const int oxm = o0 - (hxm ? ldx : 0), oxp = o0 + (hxp ? ldx : 0);
    const int oym = o0 - (hym ? sy : 0), oyp = o0 + (hyp ? sy : 0);
    auto issue = [&](Stage& st, int k) {
      const int kk = k < k1 ? k : k1 - 1;
      const int kn = kk + 1 < nz ? kk + 1 : kk;
      const int pk = kk * szx;
      st.zn = *reinterpret_cast<const V*>(X + (o0 + kn * szx));
      st.xm = *reinterpret_cast<const V*>(X + (oxm + pk));
      st.xp = *reinterpret_cast<const V*>(X + (oxp + pk));
      st.ym = *reinterpret_cast<const V*>(X + (oym + pk));
      st.yp = *reinterpret_cast<const V*>(X + (oyp + pk));
      st.ve = veff[col + nxy * kk];
    };
    V cm = *reinterpret_cast<const V*>(X + (o0 + (k0 > 0 ? k0 - 1 : k0) * szx));
    V cc = *reinterpret_cast<const V*>(X + (o0 + k0 * szx));
    Stage st[kHxPlainDepth];
#pragma unroll
    for (int s = 0; s < kHxPlainDepth; ++s) issue(st[s], k0 + s);
#pragma unroll
    for (int u = 0; u < kRun; ++u) {
      const int k = k0 + u;
      Stage& cur = st[u % kHxPlainDepth];
      const bool kok = live && k < k1;  // k < k1 is uniform over the wavefront
      const bool zmok = kok && k > 0, zpok = kok && k + 1 < nz;
      V wv;
#pragma unroll
      for (int e = 0; e < kW; ++e) {
        const double z0 = kok ? hx_elem<T, kW>(cc, e) : 0.0;
        const double nb = (hxm && kok ? hx_elem<T, kW>(cur.xm, e) : 0.0) +
                          (hxp && kok ? hx_elem<T, kW>(cur.xp, e) : 0.0) +
                          (hym && kok ? hx_elem<T, kW>(cur.ym, e) : 0.0) +
                          (hyp && kok ? hx_elem<T, kW>(cur.yp, e) : 0.0) +
                          (zmok ? hx_elem<T, kW>(cm, e) : 0.0) +
                          (zpok ? hx_elem<T, kW>(cur.zn, e) : 0.0);
        const double lx = (6.0 * z0 - nb) * ih2;
        const T o = (T)(scale * (0.5 * lx + cur.ve * z0));
        if constexpr (kW == 1) wv = o;
        else wv[e] = o;
        if (kEnergy) kin += z0 * lx;
      }
      if (kok) *reinterpret_cast<V*>(Y + (oy + k * szy)) = wv;
      cm = cc;
      cc = cur.zn;
      if (u + kHxPlainDepth < kRun) issue(cur, k + kHxPlainDepth);
    }
  }
}

// Run length 16 when that still gives every wavefront of the launch an item, else 8.
template <typename T, bool kEnergy, int kW>
__device__ inline void hx_items(const HxArgs<T>& ka, int lb, int nblk, double& kin) {
  const int nxy = ka.gr.nx * ka.gr.ny;
  const int groups = (nxy * (ka.p / kW) + kWave - 1) / kWave;
  if (groups * ((ka.gr.nz + 15) / 16) >= nblk * (kBlock / kWave))
    hx_items_run<T, kEnergy, kW, 16>(ka, lb, nblk, kin);
  else
    hx_items_run<T, kEnergy, kW, 8>(ka, lb, nblk, kin);
}

// The Hamiltonian with the Gram blocks X^T X and X^T G of the same pass (p = 32, column
// pairs, ld = 32).  A wavefront takes 4 consecutive grid columns x 16 column pairs, so on
// every plane its lanes hold a 4-point slice of X and of G exactly as FP64 MFMA fragments
// with the grid points as the contraction index: lane l holds point l / 16, columns
// 2 (l % 16) + e.  The even and odd columns form two 16-column tiles each, so X^T G and
// X^T X are 4 + 4 tiles per plane (entry (m, n) of tile (a, b) is column pair
// (2 m + a, 2 n + b)).
//
// A work item is such a 4-column slice over a run of kRun consecutive planes (16, or 8 on
// grids too small to give every wavefront an item), marched plane by plane with a software
// pipeline kHxDepth planes deep: the loads of plane k + kHxDepth (its centre values one
// plane further, its four in-plane neighbours and the two potentials) are issued while
// plane k is computed, so a wavefront never waits for one plane's loads before it can issue
// the next.  The run is unrolled completely (no register is carried around a loop, so no
// copy has to wait for a load); the pipeline drains once per item.  The z neighbours come
// from registers.  Items are ordered run-major, and blocks are remapped so that each XCD
// owns a contiguous range of items: at 64^3 one XCD holds 16 rows x 32 planes, so most
// halo rows and planes are read from its own L2.  Lanes past the grid and planes past the
// grid contribute zeros; all control flow is uniform over the wavefront (MFMAs need every
// lane).
struct HxGramAcc {
  d4 xg[4], xx[4];  // tiles (a, b) at index 2 a + b; xx[2] = xx[1]^T is not formed
};

constexpr int kHxDepth = 3;

template <typename T, int kRun>
__device__ inline void hx_gram_items(const HxArgs<T>& ka, int lb, int nblk, double& kin,
                                     HxGramAcc& g) {
  constexpr int ld = 32;
  typedef typename HxVec<T, 2>::type V2;
  const T* __restrict__ X = ka.X;
  T* __restrict__ Y = ka.Y;
  const double* __restrict__ veff = ka.veff;
  const Grid gr = ka.gr;
  const int nx = gr.nx, ny = gr.ny, nz = gr.nz;
  const int nxy = nx * ny;
  const int groups = (nxy + 3) / 4;
  const int items = groups * ((nz + kRun - 1) / kRun);
  // element offsets fit 31 bits (n * ld < 2^31 is checked at system creation): each load is
  // the uniform base pointer plus a 32-bit lane offset and a uniform plane offset
  const int sy = nx * ld, sz = nxy * ld;
  const double ih2 = gr.inv_h2 * gr.mu, scale = ka.scale;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int c = 2 * (lane % 16), q = lane / 16;
  const int nwaves = nblk * (kBlock / kWave);
  struct Stage {
    V2 zn, xm, xp, ym, yp;  // centre of plane k + 1; in-plane neighbours of plane k
    double ve;              // V_eff at plane k
  };
  for (int it = lb * (kBlock / kWave) + w; it < items; it += nwaves) {
    const int zc = it / groups, grp = it - zc * groups;
    const int col = grp * 4 + q;
    const bool live = col < nxy;
    const int colc = live ? col : 0;
    const int i = colc % nx, j = colc / nx;
    const int k0 = zc * kRun, k1 = min(k0 + kRun, nz);
    const int o0 = colc * ld + c;
    const bool hxm = live && i > 0, hxp = live && i < nx - 1;
    const bool hym = live && j > 0, hyp = live && j < ny - 1;
    const int oxm = o0 - (hxm ? ld : 0), oxp = o0 + (hxp ? ld : 0);
    const int oym = o0 - (hym ? sy : 0), oyp = o0 + (hyp ? sy : 0);
    // loads of output plane k (clamped to valid planes; masked where they are used)
    auto issue = [&](Stage& st, int k) {
      const int kk = k < k1 ? k : k1 - 1;
      const int kn = kk + 1 < nz ? kk + 1 : kk;
      const int pk = kk * sz;
      st.zn = *reinterpret_cast<const V2*>(X + (o0 + kn * sz));
      st.xm = *reinterpret_cast<const V2*>(X + (oxm + pk));
      st.xp = *reinterpret_cast<const V2*>(X + (oxp + pk));
      st.ym = *reinterpret_cast<const V2*>(X + (oym + pk));
      st.yp = *reinterpret_cast<const V2*>(X + (oyp + pk));
      st.ve = veff[colc + nxy * kk];
    };
    V2 cm = *reinterpret_cast<const V2*>(X + (o0 + (k0 > 0 ? k0 - 1 : k0) * sz));
    V2 cc = *reinterpret_cast<const V2*>(X + (o0 + k0 * sz));
    Stage st[kHxDepth];
#pragma unroll
    for (int s = 0; s < kHxDepth; ++s) issue(st[s], k0 + s);
#pragma unroll
    for (int u = 0; u < kRun; ++u) {
      const int k = k0 + u;
      Stage& cur = st[u % kHxDepth];
      const bool kok = live && k < k1;  // k < k1 is uniform over the wavefront
      const bool zmok = kok && k > 0, zpok = kok && k + 1 < nz;
      double xo[2], go[2];
      V2 wv;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const double z0 = kok ? (double)cc[e] : 0.0;
        const double nb = (hxm && kok ? (double)cur.xm[e] : 0.0) +
                          (hxp && kok ? (double)cur.xp[e] : 0.0) +
                          (hym && kok ? (double)cur.ym[e] : 0.0) +
                          (hyp && kok ? (double)cur.yp[e] : 0.0) +
                          (zmok ? (double)cm[e] : 0.0) + (zpok ? (double)cur.zn[e] : 0.0);
        const double lx = (6.0 * z0 - nb) * ih2;
        const T o = (T)(scale * (0.5 * lx + cur.ve * z0));
        wv[e] = o;
        kin += z0 * lx;
        xo[e] = z0;
        go[e] = kok ? (double)o : 0.0;
      }
      if (kok) *reinterpret_cast<V2*>(Y + (o0 + k * sz)) = wv;
#pragma unroll
      for (int ea = 0; ea < 2; ++ea)
#pragma unroll
        for (int eb = 0; eb < 2; ++eb) {
          g.xg[2 * ea + eb] = __builtin_amdgcn_mfma_f64_16x16x4f64(xo[ea], go[eb],
                                                                    g.xg[2 * ea + eb], 0, 0, 0);
          if (ea <= eb)  // X^T X is symmetric: tile (1, 0) is tile (0, 1) transposed
            g.xx[2 * ea + eb] = __builtin_amdgcn_mfma_f64_16x16x4f64(xo[ea], xo[eb],
                                                                      g.xx[2 * ea + eb], 0, 0, 0);
        }
      cm = cc;
      cc = cur.zn;
      if (u + kHxDepth < kRun) issue(cur, k + kHxDepth);
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
  double kin = 0.0;
  if constexpr (kGram) {
    __shared__ double red[3 * 4 * kWave];
    HxGramAcc g;
#pragma unroll
    for (int q = 0; q < 4; ++q) g.xg[q] = g.xx[q] = d4{0.0, 0.0, 0.0, 0.0};
    if (ka.zrun == 16)
      hx_gram_items<T, 16>(ka, lb, ks_nb, kin, g);
    else
      hx_gram_items<T, 8>(ka, lb, ks_nb, kin, g);
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      hx_reduce_tile(g.xg[q], red, w, lane);
      if (q != 2) hx_reduce_tile(g.xx[q], red, w, lane);
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
          o1[row * pp + col] = g.xg[q][r];
          if (q == 2) continue;
          o0[row * pp + col] = g.xx[q][r];
          if (q == 1) o0[col * pp + row] = g.xx[q][r];  // tile (1, 0)
        }
      }
    }
  } else {
    constexpr uintptr_t kAl = 2 * sizeof(T) - 1;
    const bool vec = ((ka.p | ka.ldx | ka.ldy) & 1) == 0 &&
                     ((reinterpret_cast<uintptr_t>(ka.X) | reinterpret_cast<uintptr_t>(ka.Y)) &
                      kAl) == 0;
    if (vec)
      hx_items<T, kEnergy, 2>(ka, lb, ks_nb, kin);
    else
      hx_items<T, kEnergy, 1>(ka, lb, ks_nb, kin);
  }
  if (kEnergy) {
    kin = block_sum(kin, sh);
    write_partial(ka.pt, SL_KIN, lb, kin);
  }
}

// (three wavefronts per SIMD without the energy partials, two with them: the register
// budgets in which the compiler keeps the pipelined loads without spilling)
template <typename T, bool kEnergy, bool kGram = false>
__global__ __launch_bounds__(256, kEnergy ? 2 : 3) void k_hx(HxArgs<T> ka) {
  k_hx_body<T, kEnergy, kGram>(ka, blockIdx.x, gridDim.x);
}

template <typename T, bool kEnergy, bool kGram = false>
__global__ __launch_bounds__(256, kEnergy ? 2 : 3) void k_hx_batch(BatchPtrs<HxArgs<T>> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_hx_body<T, kEnergy, kGram>(batch_arg(b, s), blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}

// The Gram-fused forms at two wavefronts per SIMD (at most 256 registers per lane): the
// launch holds at most 512 blocks, so that is all the occupancy there is, and the register
// budget bounds how far ahead the compiler hoists the pipelined loads.
template <typename T>
__global__ __launch_bounds__(256, 2) void k_hx_gram(HxArgs<T> ka) {
  k_hx_body<T, true, true>(ka, blockIdx.x, gridDim.x);
}

template <typename T>
__global__ __launch_bounds__(256, 2) void k_hx_gram_batch(BatchPtrs<HxArgs<T>> b) {
  const int s = batch_system(b.off, b.S, blockIdx.x);
  k_hx_body<T, true, true>(batch_arg(b, s), blockIdx.x - b.off[s], b.off[s + 1] - b.off[s]);
}


// ---- GNH pseudopotential ----------------------------------------------------------------
// V(r) = -(2/pi) int_0^inf sinc(r t) [(Z - A R_p) cos(R_p t) + A sin(R_p t)/t]
//                exp(-(t/R_c)^6) dt  (Section 4.2; the electron-ion attraction, tending to
// -Z/r), R_p = 1.15, R_c = 3.5, A = 0.1107.  It is linear in Z:  V = -[(Z - A R_p) T1 +
// A T2] with the Z-free radial integrals T1, T2 (the 2/pi included), tabulated once on
// r = 0, dr, ..., 20 bohr (dr = 1/2000) by composite Gauss-Legendre quadrature on t in
// [0, 8] (128 panels of 32 nodes; exp(-(8/3.5)^6) < 1e-61) and interpolated by cubic
// Lagrange polynomials (T1, T2 are even in r, which gives the points left of r = 0).
// Beyond the table the potential is -Z/r (the difference is below 1e-14 there).
constexpr double kGnhRp = 1.15, kGnhRc = 3.5, kGnhA = 0.1107;
constexpr int kGnhPanels = 128, kGnhNodes = 32, kGnhN = 40001;
constexpr double kGnhDr = 1.0 / 2000.0, kGnhTmax = 8.0;

struct GaussLegendre32 {
  double x[kGnhNodes], w[kGnhNodes];
};

__global__ void k_gnh_table(double* __restrict__ tab, GaussLegendre32 gl) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kGnhN) return;
  const double r = j * kGnhDr;
  const double hp = 0.5 * kGnhTmax / kGnhPanels;
  double t1 = 0.0, t2 = 0.0;
  for (int pn = 0; pn < kGnhPanels; ++pn) {
    const double mid = (2 * pn + 1) * hp;
    for (int q = 0; q < kGnhNodes; ++q) {
      const double t = mid + hp * gl.x[q], w = hp * gl.w[q];
      const double rt = r * t;
      const double sinc = rt > 0.0 ? sin(rt) / rt : 1.0;
      const double u = t / kGnhRc, u2 = u * u;
      const double e = exp(-(u2 * u2 * u2));
      t1 += w * sinc * cos(kGnhRp * t) * e;
      t2 += w * sinc * (sin(kGnhRp * t) / t) * e;
    }
  }
  tab[j] = (2.0 / kPi) * t1;
  tab[kGnhN + j] = (2.0 / kPi) * t2;
}

__global__ void k_vext_gnh(double* __restrict__ v, const double* __restrict__ R,
                           const double* __restrict__ Z, int M, Grid g,
                           const double* __restrict__ tab) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.n) return;
  const int i = idx % g.nx, j = (idx / g.nx) % g.ny, k = idx / (g.nx * g.ny);
  const double x = g.lo[0] + (i + 1) * g.h, y = g.lo[1] + (j + 1) * g.h,
               z = g.lo[2] + (k + 1) * g.h;
  const double rmax = (kGnhN - 3) * kGnhDr;
  double acc = 0.0;
  for (int a = 0; a < M; ++a) {
    const double dx = x - R[3 * a], dy = y - R[3 * a + 1], dz = z - R[3 * a + 2];
    const double d = sqrt(dx * dx + dy * dy + dz * dz);
    const double Za = Z[a];
    if (d >= rmax) {
      acc -= Za / d;
      continue;
    }
    const double u = d / kGnhDr;
    const int j0 = (int)u;
    const double f = u - j0;
    const int jm = j0 > 0 ? j0 - 1 : 1;  // T(-dr) = T(dr)
    const double wm = -f * (f - 1.0) * (f - 2.0) / 6.0, w0 = (f + 1.0) * (f - 1.0) * (f - 2.0) / 2.0,
                 w1 = -(f + 1.0) * f * (f - 2.0) / 2.0, w2 = (f + 1.0) * f * (f - 1.0) / 6.0;
    const double T1 = wm * tab[jm] + w0 * tab[j0] + w1 * tab[j0 + 1] + w2 * tab[j0 + 2];
    const double* t2 = tab + kGnhN;
    const double T2 = wm * t2[jm] + w0 * t2[j0] + w1 * t2[j0 + 1] + w2 * t2[j0 + 2];
    acc -= (Za - kGnhA * kGnhRp) * T1 + kGnhA * T2;
  }
  v[idx] = acc;
}

// Nodes and weights of the 32-point Gauss-Legendre rule on [-1, 1]: Newton's method on the
// Legendre polynomial (three-term recurrence) from the Chebyshev-type first guesses.
GaussLegendre32 gauss_legendre32() {
  GaussLegendre32 g{};
  const int n = kGnhNodes;
  for (int i = 0; i < n; ++i) {
    double x = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    g.x[i] = x;
    g.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  return g;
}

// ---- fixed-order reduction of per-block partials: one block per slot ---------------

}  // namespace

// ---- launch wrappers ------------------------------------------------------------------

void launch_vext(double* v, const double* R, const double* Z, int M, Grid g, double rc,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_vext, dim3((g.n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, v, R, Z,
                     M, g, rc);
}

size_t gnh_table_doubles() { return 2 * (size_t)kGnhN; }

void launch_vext_gnh(double* v, const double* R, const double* Z, int M, Grid g, double* table,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_gnh_table, dim3((kGnhN + 255) / 256), dim3(256), 0, st, table,
                     gauss_legendre32());
  hipLaunchKernelGGL(k_vext_gnh, dim3((g.n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, v, R,
                     Z, M, g, table);
}

void launch_enuc(double* out, const double* R, const double* Z, int M, hipStream_t st) {
  hipLaunchKernelGGL(k_enuc, dim3(1), dim3(kBlock), 0, st, out, R, Z, M);
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

// ---- Alg. 4: carrying a block over to the uniformly refined mesh ------------------------
// Fine index I along an axis of N coarse nodes: odd I is coarse node (I - 1)/2 itself, even
// I lies half-way between coarse nodes I/2 - 1 and I/2, where -1 and N are the zero
// boundary.  One thread per (fine node, column); the up to 8 coarse values are summed in
// FP64 and rounded once.
__device__ inline int prolong_axis(int I, int N, int* i0, int* i1) {
  if (I & 1) {
    *i0 = (I - 1) >> 1;
    *i1 = -1;
    return 1;
  }
  *i0 = (I >> 1) - 1;
  *i1 = (I >> 1) < N ? (I >> 1) : -1;
  return 2;
}

template <typename T>
__global__ void k_prolong(const T* __restrict__ xc, int ldc, int cnx, int cny, int cnz,
                          T* __restrict__ xf, int ldf, int p, double scale) {
  const int fnx = 2 * cnx + 1, fny = 2 * cny + 1;
  const size_t fn = (size_t)fnx * fny * (2 * cnz + 1);
  const size_t total = fn * p;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t node = e / p;
    const int c = (int)(e - node * p);
    const int I = (int)(node % fnx), J = (int)((node / fnx) % fny), K = (int)(node / ((size_t)fnx * fny));
    int xi[2], yi[2], zi[2];
    const int nxs = prolong_axis(I, cnx, &xi[0], &xi[1]);
    const int nys = prolong_axis(J, cny, &yi[0], &yi[1]);
    const int nzs = prolong_axis(K, cnz, &zi[0], &zi[1]);
    const double wx = nxs == 1 ? 1.0 : 0.5, wy = nys == 1 ? 1.0 : 0.5, wz = nzs == 1 ? 1.0 : 0.5;
    double acc = 0.0;
    for (int a = 0; a < nzs; ++a) {
      if (zi[a] < 0) continue;
      for (int b = 0; b < nys; ++b) {
        if (yi[b] < 0) continue;
        for (int d = 0; d < nxs; ++d) {
          if (xi[d] < 0) continue;
          const size_t g = (size_t)xi[d] + (size_t)cnx * ((size_t)yi[b] + (size_t)cny * zi[a]);
          acc += (double)xc[g * ldc + c];
        }
      }
    }
    xf[node * ldf + c] = (T)(scale * wx * wy * wz * acc);
  }
}

template <typename T>
void launch_prolong(const T* xc, int ldc, int cnx, int cny, int cnz, T* xf, int ldf, int p,
                    double scale, hipStream_t st) {
  const size_t total = (size_t)(2 * cnx + 1) * (2 * cny + 1) * (2 * cnz + 1) * p;
  const size_t want = (total + kBlock - 1) / kBlock;
  const unsigned nb = (unsigned)(want < 65536 ? (want < 1 ? 1 : want) : 65536);
  hipLaunchKernelGGL(k_prolong<T>, dim3(nb), dim3(kBlock), 0, st, xc, ldc, cnx, cny, cnz, xf,
                     ldf, p, scale);
}
template void launch_prolong<double>(const double*, int, int, int, int, double*, int, int,
                                     double, hipStream_t);
template void launch_prolong<float>(const float*, int, int, int, int, float*, int, int, double,
                                    hipStream_t);

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
               int use_h, int use_x, const CgState* cg, Partials pt, hipStream_t st,
               bool cg_check, const double* vbc) {
  hipLaunchKernelGGL(k_xc, dim3(scalar_blocks(g.n)), dim3(kBlock), 0, st,
                     XcArgs{rho, vh, vext, veff, g, use_h, use_x, cg, pt, cg_check ? 1 : 0,
                            vbc});
}

// ---- monopole boundary of the Hartree potential -----------------------------------------
__device__ inline double bc_value(const Grid& g, int i, int j, int k, double Q, double cx,
                                  double cy, double cz) {
  const double dx = g.lo[0] + (i + 1) * g.h - cx, dy = g.lo[1] + (j + 1) * g.h - cy,
               dz = g.lo[2] + (k + 1) * g.h - cz;
  return Q / sqrt(dx * dx + dy * dy + dz * dz);
}

__global__ void k_bc_rhs(double* __restrict__ out, Grid g, double Q, double cx, double cy,
                         double cz) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.n) return;
  const int i = idx % g.nx, j = (idx / g.nx) % g.ny, k = idx / (g.nx * g.ny);
  double acc = 0.0;
  if (i == 0 || j == 0 || k == 0 || i == g.nx - 1 || j == g.ny - 1 || k == g.nz - 1) {
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int a = i + dx, b = j + dy, c = k + dz;
          if (a >= 0 && a < g.nx && b >= 0 && b < g.ny && c >= 0 && c < g.nz) continue;
          const int cls = (dx != 0) + (dy != 0) + (dz != 0);
          double w = 0.0;
          if (!g.q1) w = cls == 1 ? g.inv_h2 : 0.0;
          else w = cls == 2 ? g.h / 6.0 : (cls == 3 ? g.h / 12.0 : 0.0);
          if (w != 0.0) acc += w * bc_value(g, a, b, c, Q, cx, cy, cz);
        }
  }
  out[idx] = acc / (4.0 * kPi * g.rhs_scale);
}

__global__ void k_bc_point(const double* __restrict__ v, Grid g, double Q, double cx,
                           double cy, double cz, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double ux = (cx - g.lo[0]) / g.h - 1.0, uy = (cy - g.lo[1]) / g.h - 1.0,
               uz = (cz - g.lo[2]) / g.h - 1.0;
  const int bx = (int)floor(ux), by = (int)floor(uy), bz = (int)floor(uz);
  const double tx = ux - bx, ty = uy - by, tz = uz - bz;
  double acc = 0.0;
  for (int dk = 0; dk < 2; ++dk)
    for (int dj = 0; dj < 2; ++dj)
      for (int di = 0; di < 2; ++di) {
        const int i = bx + di, j = by + dj, k = bz + dk;
        const double w = (di ? tx : 1.0 - tx) * (dj ? ty : 1.0 - ty) * (dk ? tz : 1.0 - tz);
        const bool in = i >= 0 && i < g.nx && j >= 0 && j < g.ny && k >= 0 && k < g.nz;
        const double val = in ? v[i + g.nx * (j + g.ny * k)] : bc_value(g, i, j, k, Q, cx, cy, cz);
        acc += w * val;
      }
  *out = -0.5 * Q * acc;
}

void launch_bc_rhs(double* out, Grid g, double Q, double cx, double cy, double cz,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_bc_rhs, dim3((g.n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, out, g, Q,
                     cx, cy, cz);
}

void launch_bc_point(const double* v, Grid g, double Q, double cx, double cy, double cz,
                     double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_bc_point, dim3(1), dim3(kWave), 0, st, v, g, Q, cx, cy, cz, out);
}

template <typename T>
void launch_hx(const T* X, int ldx, T* Y, int ldy, const double* veff,
               Grid g, int p, double scale, Partials* pt, double* gram_part, hipStream_t st) {
  if (gram_part) {
    hipLaunchKernelGGL((k_hx_gram<T>), dim3(hx_gram_blocks(g.n)), dim3(kBlock), 0, st,
                       HxArgs<T>{X, ldx, Y, ldy, veff, g, p, scale, *pt, gram_part,
                                 hx_zrun_of(g)});
    return;
  }
  const int nb = hx_blocks(g.n, p);
  if (pt) {
    hipLaunchKernelGGL((k_hx<T, true>), dim3(nb), dim3(kBlock), 0, st,
                       HxArgs<T>{X, ldx, Y, ldy, veff, g, p, scale, *pt, nullptr});
  } else {
    Partials none{nullptr, 0};
    hipLaunchKernelGGL((k_hx<T, false>), dim3(nb), dim3(kBlock), 0, st,
                       HxArgs<T>{X, ldx, Y, ldy, veff, g, p, scale, none, nullptr});
  }
}
template void launch_hx<double>(const double*, int, double*, int, const double*, Grid, int,
                                double, Partials*, double*, hipStream_t);
template void launch_hx<float>(const float*, int, float*, int, const double*, Grid, int, double,
                               Partials*, double*, hipStream_t);

int hx_blocks(int n, int p) { return stream_blocks((size_t)n * p / (2 * kHxChunk) + 1); }

// Blocks of the Hamiltonian that also forms the Gram blocks of [X, G]: as many as the Gram
// launch would use (each block writes one partial tile set).
int hx_gram_blocks(int n) {
  const int c = (n + 63) / 64;
  return c < 1 ? 1 : (c > 512 ? 512 : c);
}

bool hx_fuses_gram(int p) { return p == 32; }

// Planes per work item of the Gram-fused Hamiltonian: 16, or 8 when runs of 16 would leave
// wavefronts of its hx_gram_blocks(n) blocks without an item.
int hx_zrun_of(const Grid& g) {
  return (g.hx_zrun == 8 || g.hx_zrun == 16) ? g.hx_zrun : hx_zrun(g.nx * g.ny, g.nz);
}

int hx_zrun(int nxy, int nz) {
  const int groups = (nxy + 3) / 4;
  const int waves = hx_gram_blocks(nxy * nz) * (kBlock / kWave);
  return groups * ((nz + 15) / 16) >= waves ? 16 : 8;
}


void launch_xc_batch(const BatchPtrs<XcArgs>& b, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_xc_batch, dim3(blocks), dim3(kBlock), 0, st, b);
}

template <typename T>
void launch_hx_batch(const BatchPtrs<HxArgs<T>>& b, int blocks, bool gram, hipStream_t st) {
  if (gram)
    hipLaunchKernelGGL((k_hx_gram_batch<T>), dim3(blocks), dim3(kBlock), 0, st, b);
  else
    hipLaunchKernelGGL((k_hx_batch<T, true>), dim3(blocks), dim3(kBlock), 0, st, b);
}
template void launch_hx_batch<double>(const BatchPtrs<HxArgs<double>>&, int, bool,
                                      hipStream_t);
template void launch_hx_batch<float>(const BatchPtrs<HxArgs<float>>&, int, bool, hipStream_t);

}  // namespace ks
