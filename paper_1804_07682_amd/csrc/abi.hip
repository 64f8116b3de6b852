// Status codes, error messages and small ABI queries of libgna_hip.so.
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "gna_internal.h"

namespace gna {

static thread_local char g_last_error[512] = "";

// Pending injected failures (gna_debug_inject_hip_errors): each successful
// HIP status checked by the library while this is positive is reported as a
// failure instead, and the count goes down by one.
static std::atomic<int> g_inject_hip{0};

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return code;
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) {
    int n = g_inject_hip.load();
    while (n > 0 && !g_inject_hip.compare_exchange_weak(n, n - 1)) {
    }
    if (n > 0) return fail(GNA_E_HIP, "%s: injected failure (gna_debug_inject_hip_errors)", what);
    return GNA_OK;
  }
  return fail(GNA_E_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

void clear_error() { g_last_error[0] = '\0'; }

}  // namespace gna

extern "C" {

int gna_abi_version(void) { return GNA_ABI_VERSION; }

const char* gna_strerror(int status) {
  switch (status) {
    case GNA_OK: return "ok";
    case GNA_E_INVAL: return "invalid argument";
    case GNA_E_DOMAIN: return "domain error latched on the device";
    case GNA_E_HIP: return "HIP runtime error";
    case GNA_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case GNA_E_UNSUPPORTED: return "unsupported request";
    default: return "unknown status";
  }
}

const char* gna_last_error_message(void) { return gna::g_last_error; }

int gna_debug_inject_hip_errors(int32_t count) {
  gna::clear_error();
  if (count < 0) return gna::fail(GNA_E_INVAL, "gna_debug_inject_hip_errors: count %d < 0", count);
  gna::g_inject_hip.store(count);
  return GNA_OK;
}

int32_t gna_debug_pending_hip_errors(void) { return gna::g_inject_hip.load(); }

}  // extern "C"
