// Host-side helpers shared by the library's translation units (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.h"

namespace smx {

// Records a message for strassen_last_error and returns `code`.
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
void clear_error();

#define SMX_HIP(call)                                      \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return smx::hip_fail(e_, #call); \
  } while (0)

// The kNumTables operation tables (host copies; the device copies are uploaded per device).
const TableDev* host_tables();
// Current device checked (gfx950) and its constant tables uploaded; returns 0 or an error code.
int device_ready(int* dev_out);

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return cdiv(a, b) * b; }

}  // namespace smx
