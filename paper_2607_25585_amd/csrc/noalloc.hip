// Allocation-free start vectors: ftlm_gaussian_vectors_noalloc.
//
// The start kernel of ftlm_gaussian_vectors writes per-block norm partials and
// the column norms next to the vectors it generates.  ftlm_gaussian_vectors
// keeps a private buffer for them that it allocates on its first call on a
// device; this variant takes that memory from a file-scope device array, so it
// never calls hipMalloc, hipFree or an allocating library routine (callers under
// HIP graph capture or in loops that must not allocate).
//
// The array holds the partials of at most kNaBlocks blocks for kNaCols columns.
// Each GPU has its own copy at its own address, obtained once per device with
// hipGetSymbolAddress and kept for the life of the process; host code uses that
// address only, never the array's name.  Every call on one GPU shares the
// array: calls that overlap on one GPU race on the partials (the vectors they
// write are unaffected, since the partials only feed the discarded norms).
// Nothing in the array needs to start at zero: the partials are written with
// plain stores before they are read, within each call.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ftlm_internal.hpp"

namespace ftlm {
namespace {

constexpr int kNaBlocks = 2048;  // grid cap of the start kernel in this entry point
constexpr int kNaCols = 64;      // columns per call (the ABI's maximum)
constexpr size_t kNaPart = (size_t)kNaBlocks * kNaCols;  // doubles of the partials
constexpr size_t kNaWords = kNaPart + kNaCols + 64;      // + inverse norms + counter words

static __device__ __align__(256) double scratch[kNaWords];

constexpr int kNaMaxDev = 64;
std::mutex g_na_mu;
double *g_na_ptr[kNaMaxDev] = {};

// Device address of this GPU's copy of the array (looked up once per device,
// with that device current).
int scratch_address(double **out, std::string &err) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    err = "hipGetDevice failed";
    return FTLM_EHIP;
  }
  if (dev < 0 || dev >= kNaMaxDev) {
    err = "device index out of range";
    return FTLM_ERANGE;
  }
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_na_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      err = std::string("hipGetSymbolAddress of the start-vector scratch failed: ") + hipGetErrorString(e);
      return FTLM_EHIP;
    }
    g_na_ptr[dev] = reinterpret_cast<double *>(p);
  }
  *out = g_na_ptr[dev];
  return FTLM_OK;
}

}  // namespace
}  // namespace ftlm

using namespace ftlm;

extern "C" int ftlm_gaussian_vectors_noalloc(uint64_t seed, uint32_t instance, uint32_t field, uint32_t r0,
                                             int32_t n_cols, uint64_t dim, void *out, void *stream) {
  if (!out) { set_error("out is NULL"); return FTLM_EINVAL; }
  if (n_cols < 1 || n_cols > kNaCols) {
    set_error("n_cols must be in [1, 64] (the scratch array holds the partials of 64 columns)");
    return FTLM_ERANGE;
  }
  if (dim < 1 || dim >= (1ull << 32)) { set_error("dim out of range"); return FTLM_ERANGE; }
  std::string err;
  double *base = nullptr;
  const int rc0 = scratch_address(&base, err);
  if (rc0) { set_error(err); return rc0; }
  double *part = base;                 // [blocks <= kNaBlocks][n_cols]
  double *sx0 = base + kNaPart;        // [n_cols]
  unsigned *counter = reinterpret_cast<unsigned *>(base + kNaPart + kNaCols);
  const int rc = launch_gaussian(seed, instance, field, r0, n_cols, (uint32_t)dim, FTLM_C128, out, part,
                                 counter, sx0, kNaBlocks, (hipStream_t)stream);
  if (rc) set_error("gaussian launch failed");
  return rc;
}
