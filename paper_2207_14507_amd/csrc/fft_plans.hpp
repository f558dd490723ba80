// Radix plans of the transform lengths the library is built for.  Row transforms run
// on pairs of real rows packed into one complex row (length N = frame width); column
// transforms run on the packed half spectrum (length M = frame height).
#pragma once

#include "fft_device.hpp"

namespace prnu {

#define PRNU_PLAN(L, ...)                                   \
  template <>                                               \
  struct PlanFor<L> {                                       \
    using RS = Radices<__VA_ARGS__>;                        \
    static_assert(RS::product() == L, "plan must factor L"); \
  };

PRNU_PLAN(64, 8, 8)
PRNU_PLAN(96, 8, 12)
PRNU_PLAN(120, 8, 15)
PRNU_PLAN(160, 10, 16)
PRNU_PLAN(256, 16, 16)
PRNU_PLAN(720, 16, 9, 5)
PRNU_PLAN(1080, 8, 9, 15)
PRNU_PLAN(1280, 16, 16, 5)
PRNU_PLAN(1920, 16, 12, 10)
PRNU_PLAN(2160, 16, 9, 15)
PRNU_PLAN(3840, 16, 16, 15)

#undef PRNU_PLAN

// X-macro lists of supported lengths: every planned length can be a row length (frame
// width N); column lengths (frame height M) are limited by the LDS of one column strip.
#define PRNU_FOR_EACH_LENGTH(X) \
  X(64) X(96) X(120) X(160) X(256) X(720) X(1080) X(1280) X(1920) X(2160) X(3840)
#define PRNU_FOR_EACH_COL_LENGTH(X) \
  X(64) X(96) X(120) X(160) X(256) X(720) X(1080) X(1280) X(1920) X(2160)

}  // namespace prnu
