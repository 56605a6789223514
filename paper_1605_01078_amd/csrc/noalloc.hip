// strassen_dgemm_noalloc: strassen_dgemm for callers that cannot allocate device memory.
//
// Its workspace is a file-scope device array, `scratch`, of kScratchBytes, held by every device
// the library runs on until the process ends.  The host never uses the array's name as an
// address (in host code it names a host-side stand-in): the first call on a device resolves the
// device address with hipGetSymbolAddress, with that device current, and keeps it per device.
// The call then runs exactly what strassen_dgemm runs with that buffer as a caller workspace:
// AB and Naive keep their temporaries there (sizes beyond the scratch are refused); ABC uses it
// for block-padded copies and staged sums only where they fit, and otherwise takes its
// workspace-free path, as with any workspace too small.  Nothing in the scratch has to start at
// zero: every kernel that reads a workspace element (padded copies, staged sums, product
// temporaries, operand-sum temporaries) reads only elements an earlier kernel of the same call
// wrote.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "../../include/strassen.h"
#include "internal.h"

namespace smx {

constexpr size_t kScratchBytes = size_t(256) << 20;   // STRASSEN_NOALLOC_SCRATCH_BYTES
static_assert(kScratchBytes == STRASSEN_NOALLOC_SCRATCH_BYTES, "header and library agree");

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_ptr;   // device address of `scratch`, per device

// Device address of this device's scratch array (resolved once per device, with it current).
static int scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(STRASSEN_ERR_HIP, "hipGetSymbolAddress(scratch) gave NULL");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

}  // namespace smx

extern "C" int strassen_dgemm_noalloc(int64_t m, int64_t n, int64_t k, double alpha,
                                      const double* A, int64_t lda, const double* B, int64_t ldb,
                                      double beta, double* C, int64_t ldc, int levels,
                                      int variant, void* stream) {
  smx::WsSource ws;
  ws.fixed = true;
  ws.bytes = smx::kScratchBytes;
  ws.what = "the static scratch of strassen_dgemm_noalloc";
  ws.resolve = smx::scratch_address;   // first use on a device, with that device current
  return smx::dgemm(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, levels, variant, ws,
                    static_cast<hipStream_t>(stream));
}
