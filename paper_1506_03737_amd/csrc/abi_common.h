// Helpers shared by the C-ABI source files of liblpc: the thread-local error detail, HIP error checks that unwind to
// the entry point, and the guard that turns any exception into a status code (no exception crosses the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <exception>
#include <string>

#include "../../include/lpc.h"

namespace lpc {
namespace abi {

// Records a printf-style detail for lpc_last_error() and returns s.
lpc_status fail(lpc_status s, const char* fmt, ...);
const char* last_error();

struct HipError {
  hipError_t e;
  const char* what;
};

inline void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipError{e, what};
}

template <class F>
lpc_status guarded(F body) {
  try {
    return body();
  } catch (const HipError& e) {
    return fail(LPC_ERR_HIP, "%s failed: %s", e.what, hipGetErrorString(e.e));
  } catch (const std::exception& e) {
    return fail(LPC_ERR_HIP, "internal error: %s", e.what());
  } catch (...) {
    return fail(LPC_ERR_HIP, "unknown internal error");
  }
}

}  // namespace abi
}  // namespace lpc
