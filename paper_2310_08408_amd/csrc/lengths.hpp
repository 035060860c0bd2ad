// Every transform length the library uses, with its compile-time radix
// schedule (largest radix first).  Requested sizes are rounded up to the
// next length in this list, which is exact for zero-padded convolution and
// for Bluestein.  X(n, radices...).  Host-only: included by the device
// engine and by the host-side validation.
#pragma once

#define LP_LENGTHS(X)                                                                            \
  X(1, 1) X(2, 2) X(4, 4) X(8, 8) X(16, 16) X(32, 8, 4) X(64, 8, 8) X(96, 12, 8) X(128, 16, 8)  \
  X(192, 16, 12) X(256, 16, 16) X(384, 8, 8, 6) X(512, 8, 8, 8) X(768, 12, 8, 8)                \
  X(1024, 16, 8, 8) X(1536, 16, 12, 8) X(2048, 16, 8, 16) X(3072, 16, 16, 12)                   \
  X(4096, 16, 16, 16) X(6144, 32, 16, 12) X(8192, 32, 16, 16)

// Alternative schedules the autotuner may choose for a length (FP32 only):
// equal first and last radices, so that the convolution passes keep the
// spectrum product in registers and the column passes can run
// persistently.  A schedule changes rounding, so a tuned choice is fixed per
// plan (or tuned shape) and recorded.  X(n, radices...)
#define LP_ALT_LENGTHS(X) X(768, 8, 12, 8) X(1024, 8, 16, 8) X(1536, 16, 6, 16) X(3072, 16, 12, 16)

namespace lp {
constexpr int kMaxLen = 8192;
}  // namespace lp
