// Radix plans of the transform lengths the library is built for.
//
// Row plans run on pairs of real rows packed into one complex row (length N = frame
// width), one transform per workgroup of 64 threads (128 for widths 1280 and 1920, 256
// for 3840); the first radix is chosen so that the first pass maps one butterfly onto
// each thread.  Column plans run on strips of 8 interleaved columns of the packed half
// spectrum (length M = frame height) with 256 threads (512 for 720 and 1080; from 1280
// rows on, each 4-column half of a strip on 256 or 512 threads); their radices keep most
// lanes busy with few butterflies per thread.  At 1080 and 2160 rows the plans were
// picked by timing the alternatives on the device: an odd last radix (the inverse
// transform's first, whose stores a radix apart then fall on distinct LDS banks; at 1080
// rows an odd first radix too) with a large middle radix beats the plans that keep every
// pass fullest (9 x 24 x 5 is 7% faster than 18 x 6 x 10, 12 x 20 x 9 is 12% faster than
// 18 x 6 x 20).  As prime-factor plans (no twiddle loads or multiplies; the column
// kernel reads the rows of dimension 0 in the Ruritanian order), 1080 = 27 x 8 x 5 is
// 8% faster again than 9 x 24 x 5 and 720 = 16 x 9 x 5 10% faster than 12 x 12 x 5
// (9 x 16 x 5 and 5 x 16 x 9 lie between); at 2160 rows the prime-factor plans
// 27 x 16 x 5 and 16 x 27 x 5 lose to 12 x 20 x 9.  The inverse column transform uses the
// reversed column plan, so that its first pass consumes the forward transform's
// last-pass registers directly.
#pragma once

#include "fft_device.hpp"

namespace prnu {

template <int L>
struct RowPlan;
template <int L>
struct ColPlan;

#define PRNU_PLAN(KIND, L, ...)                              \
  template <>                                                \
  struct KIND<L> {                                           \
    using RS = Radices<__VA_ARGS__>;                         \
    static_assert(RS::product() == L, "plan must factor L"); \
    static_assert(RS::count >= 2, "at least two passes");    \
  };

// A prime-factor plan: pairwise coprime dimensions, no twiddles (Coprime above).
#define PRNU_PLAN_PFA(KIND, L, ...)                          \
  template <>                                                \
  struct KIND<L> {                                           \
    using RS = Coprime<__VA_ARGS__>;                         \
    static_assert(RS::product() == L, "plan must factor L"); \
    static_assert(RS::count >= 2, "at least two passes");    \
  };

PRNU_PLAN(RowPlan, 64, 8, 8)
PRNU_PLAN(RowPlan, 96, 12, 8)
PRNU_PLAN(RowPlan, 120, 15, 8)
PRNU_PLAN(RowPlan, 160, 10, 16)
PRNU_PLAN(RowPlan, 256, 16, 16)
PRNU_PLAN(RowPlan, 720, 12, 6, 10)
PRNU_PLAN(RowPlan, 1080, 15, 8, 9)
PRNU_PLAN(RowPlan, 1280, 10, 16, 8)
PRNU_PLAN(RowPlan, 1920, 15, 8, 16)
PRNU_PLAN(RowPlan, 2160, 15, 12, 12)
PRNU_PLAN(RowPlan, 3840, 15, 16, 16)

PRNU_PLAN(ColPlan, 64, 8, 8)
PRNU_PLAN(ColPlan, 96, 8, 12)
PRNU_PLAN(ColPlan, 120, 8, 15)
PRNU_PLAN(ColPlan, 160, 10, 16)
PRNU_PLAN(ColPlan, 256, 16, 16)
PRNU_PLAN_PFA(ColPlan, 720, 16, 9, 5)
PRNU_PLAN_PFA(ColPlan, 1080, 27, 8, 5)
PRNU_PLAN(ColPlan, 1280, 16, 8, 10)
PRNU_PLAN(ColPlan, 1920, 16, 12, 10)
PRNU_PLAN(ColPlan, 2160, 12, 20, 9)

#undef PRNU_PLAN
#undef PRNU_PLAN_PFA

// X-macro lists of supported lengths: every planned length can be a row length (frame
// width N); column lengths (frame height M) are limited by the LDS of one column strip.
#define PRNU_FOR_EACH_LENGTH(X) \
  X(64) X(96) X(120) X(160) X(256) X(720) X(1080) X(1280) X(1920) X(2160) X(3840)
#define PRNU_FOR_EACH_COL_LENGTH(X) \
  X(64) X(96) X(120) X(160) X(256) X(720) X(1080) X(1280) X(1920) X(2160)

// Which twiddle table: the row plan, the column plan, or the reversed column plan.
enum PlanKind { kRowPlan = 0, kColPlan = 1, kColPlanRev = 2 };

}  // namespace prnu
