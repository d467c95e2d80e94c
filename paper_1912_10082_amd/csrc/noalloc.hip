// The Gram-Schmidt contraction C = A^T B without device allocation.
//
// sts_gram allocates the per-chunk partial products of the contraction on
// every call.  sts_gram_noalloc runs the same kernels with those partials in
// `scratch`, a file-scope device array of kNoAllocMaxM columns' worth, so a
// caller that cannot allocate device memory can still call it.  Each device
// the library runs on holds its own copy of the array until the process ends.
// Host code never passes the array's name to a kernel: the name is a host-side
// stand-in, so the device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and kept.
//
// The kernels overwrite every partial they read, so nothing needs clearing
// between calls.  Calls that overlap on one device (other streams, other host
// threads) share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "sts_internal.h"

namespace sts {
namespace {

constexpr int kNoAllocMaxM = 512;
// The contraction splits the rows into at most 256 chunks, each holding an
// m16 x 16 block of partial products (m16 = m rounded up to 16).
constexpr int64_t kScratchDoubles = 256LL * kNoAllocMaxM * 16;   // 16 MiB

__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up on the
// first call there.
double* scratch_on_current_device() {
  int dev = 0;
  STS_HIP(hipGetDevice(&dev));
  STS_REQUIRE(dev >= 0 && dev < kMaxDevices, STS_E_DEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    STS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch[dev] = static_cast<double*>(p);
  }
  return g_scratch[dev];
}

}  // namespace
}  // namespace sts

extern "C" sts_status sts_gram_noalloc(int64_t rows, int32_t m, int32_t n, const double* A,
                                       int64_t lda, const double* B, int64_t ldb, double* C,
                                       int64_t ldc, void* stream) {
  using namespace sts;
  try {
    set_error(std::string());
    STS_REQUIRE(rows >= 0 && m >= 1 && n >= 1 && n <= 16, STS_E_INVALID, "bad sizes");
    STS_REQUIRE(m <= kNoAllocMaxM, STS_E_INVALID,
                "sts_gram_noalloc: m = " + std::to_string(m) + " exceeds the " +
                    std::to_string(kNoAllocMaxM) + " columns its device scratch holds");
    STS_REQUIRE(A && B && C && lda >= rows && ldb >= rows && ldc >= m, STS_E_INVALID,
                "bad buffers");
    STS_REQUIRE(gemm_tn_partial_size(rows > 0 ? rows : 1, m) <= kScratchDoubles, STS_E_INVALID,
                "partial products exceed the device scratch");
    double* part = scratch_on_current_device();
    gemm_tn(rows, m, n, A, lda, B, ldb, C, ldc, part, static_cast<hipStream_t>(stream));
    return STS_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (...) {
    set_error("unexpected exception");
    return STS_E_DEVICE;
  }
}
