// ks_gram_static: the Gram blocks of ks_gram for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops).  It needs no system handle and no
// workspace: the per-chunk partial products live in one file-scope device array of fixed
// size, shared by every call on a GPU.
//
// The array's name is a host-side stand-in in host code, not a device address.  Its
// device address is looked up once per device (hipGetSymbolAddress with that device
// current) and only that address reaches kernels.
#include <mutex>
#include <string>

#include "ks_common.h"

namespace {

constexpr int kStaticMaxP = 64;       // columns of A and B
constexpr int kStaticMaxChunks = 128; // row chunks of the partial products
constexpr int kStaticPP = 64;         // padded p_p of the largest block
// partials [chunk][3][pp][pp], then the reduced padded products [3][pp][pp]
constexpr size_t kPartDoubles = (size_t)kStaticMaxChunks * 3 * kStaticPP * kStaticPP;
constexpr size_t kScratchDoubles = kPartDoubles + (size_t)3 * kStaticPP * kStaticPP;
constexpr int kMaxDevices = 64;

}  // namespace

// 12.7 MB per GPU the library runs on, held until the process ends.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};
// errors are reported through ks_last_error(NULL) of the calling thread
int set_err(int code, const char* msg) {
  ks::set_thread_error(msg);
  return code;
}

// Device address of `scratch` on the current device (looked up on the first call there).
int scratch_address(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return set_err(KS_E_HIP, "no current HIP device");
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return set_err(KS_E_HIP, "hipGetSymbolAddress of the static scratch failed");
    }
    g_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_ptr[dev];
  return KS_OK;
}

}  // namespace

extern "C" int ks_gram_static(const void* A, const void* B, int n, int p, int ld,
                              int precision, double* out, void* hip_stream) {
  if (!A || !B || !out) return set_err(KS_E_INVAL, "null argument");
  if (n < 1) return set_err(KS_E_INVAL, "n must be >= 1");
  if (p < 1 || p > kStaticMaxP)
    return set_err(KS_E_INVAL, "p must be in [1, 64] for the static scratch");
  if (ld == 0) ld = p;
  if (ld < p) return set_err(KS_E_INVAL, "ld must be >= p");
  if ((double)n * ld >= 2147483647.0) return set_err(KS_E_INVAL, "n * ld must be < 2^31");
  if (precision != KS_PREC_FP64 && precision != KS_PREC_FP32 &&
      precision != KS_PREC_MIXED_BF16)
    return set_err(KS_E_INVAL, "unknown precision");
  double* base = nullptr;
  int rc = scratch_address(&base);
  if (rc) return rc;
  const bool f32 = precision != KS_PREC_FP64;
  const int pp = ks::round_up(p, 16);
  int nchunks = ks::gram_chunks(n, pp);
  if (nchunks > kStaticMaxChunks) nchunks = kStaticMaxChunks;
  double* part = base;
  double* red = base + kPartDoubles;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int all = ks::kGramAA | ks::kGramAB | ks::kGramBB;
  // every chunk writes all tiles of the three products (padding columns as zeros), and the
  // reduction writes every padded entry, so nothing in the scratch has to start at zero
  ks::launch_gram(A, B, f32, ld, n, p, all, part, nchunks, st);
  ks::launch_gram_reduce(part, nchunks, pp, all, red, nullptr, st);
  ks::launch_compact_gram(red, pp, p, out, st);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(KS_E_HIP, hipGetErrorString(e));
  return KS_OK;
}
