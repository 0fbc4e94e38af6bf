// Host utilities shared by the lattice builder and the solver: status codes,
// the per-thread error message, and layout constants.
#pragma once

#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "lbm_sparse.h"

namespace lbm {

// Nodes per GPU wavefront tile; the RIA wave tables are built for this width.
constexpr int64_t kWave = 64;
// Nodes per workgroup of the step kernels (four wavefront tiles), the unit
// of a workgroup schedule.
constexpr int64_t kGroupNodes = 256;
// XCDs of the device: the hardware deals workgroup b to XCD b mod 8.
constexpr int64_t kXcds = 8;

inline char* error_buffer() {
  static thread_local char buf[512] = {0};
  return buf;
}

inline void clear_error() { error_buffer()[0] = 0; }

inline int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(error_buffer(), 512, fmt, ap);
  va_end(ap);
  return code;
}

}  // namespace lbm
