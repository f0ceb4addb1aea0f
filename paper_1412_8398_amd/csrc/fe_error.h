// Thread-local error text shared by every C entry point of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/fe.h"

namespace fe {

inline std::string& last_error_text() {
  static thread_local std::string s;
  return s;
}

inline fe_status fail(fe_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  last_error_text() = buf;
  return st;
}

}  // namespace fe

#define HIP_TRY(expr)                                                                           \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return ::fe::fail(e_ == hipErrorOutOfMemory ? FE_ERR_OOM : FE_ERR_DEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                       \
  } while (0)
