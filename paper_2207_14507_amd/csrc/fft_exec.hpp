// Pass execution for the Stockham building blocks: LDS loads and stores of a pass's
// butterflies, their arithmetic, runs of LDS-to-LDS passes, and the host twiddle
// tables.  Kernels feed the first pass of a plan from registers (gathered or loaded
// data) and take the last pass's outputs in registers.
#pragma once

#include <cmath>
#include <vector>

#include "fft_plans.hpp"

namespace prnu {

template <class PS, int B, int T>
__device__ __forceinline__ void lds_load(const c32* buf, c32 (&v)[PS::ROUNDS][PS::R], int tid) {
#pragma unroll
  for (int r = 0; r < PS::ROUNDS; ++r) {
    const int g = tid + r * T;
    if (PS::full() || g < PS::TOT) {
      const int b = g % B, j = g / B;
#pragma unroll
      for (int q = 0; q < PS::R; ++q) v[r][q] = buf[lds_slot<B>(PS::in_el(j, q) * B + b)];
    }
  }
}

template <class PS, int B, int T>
__device__ __forceinline__ void lds_store(c32* buf, const c32 (&v)[PS::ROUNDS][PS::R], int tid) {
#pragma unroll
  for (int r = 0; r < PS::ROUNDS; ++r) {
    const int g = tid + r * T;
    if (PS::full() || g < PS::TOT) {
      const int b = g % B, j = g / B;
#pragma unroll
      for (int q = 0; q < PS::R; ++q) buf[lds_slot<B>(PS::out_el(j, q) * B + b)] = v[r][q];
    }
  }
}

template <class PS, int B, int T, bool INV>
__device__ __forceinline__ void pass_compute(c32 (&v)[PS::ROUNDS][PS::R], const c32* __restrict__ tw, int tid) {
#pragma unroll
  for (int r = 0; r < PS::ROUNDS; ++r) {
    const int g = tid + r * T;
    if (PS::full() || g < PS::TOT) PS::template butterfly<INV>(v[r], g / B, tw);
  }
}

// Passes [P, P1) of plan RS, each reading and writing LDS in place (loads, barrier,
// compute, stores, barrier; no barrier between the loads and the stores of a pass
// whose butterflies write the elements they read).  The caller has made the data
// visible before the call.
template <class RS, int P, int P1, int B, int T, bool INV>
__device__ __forceinline__ void lds_passes(c32* buf, const c32* __restrict__ tw, int tid) {
  if constexpr (P < P1) {
    using PS = Pass<RS, P, B, T>;
    c32 v[PS::ROUNDS][PS::R];
    lds_load<PS, B, T>(buf, v, tid);
    if constexpr (!PS::in_place) __syncthreads();
    pass_compute<PS, B, T, INV>(v, tw, tid);
    lds_store<PS, B, T>(buf, v, tid);
    __syncthreads();
    lds_passes<RS, P + 1, P1, B, T, INV>(buf, tw, tid);
  }
}

// One LDS-to-LDS pass whose twiddles come from a table of its own (entry
// k (R - 1) + q - 1 = W_{Ns R}^{k q}), e.g. a copy in LDS.
template <class PS, int B, int T, bool INV>
__device__ __forceinline__ void lds_pass_own(c32* buf, const c32* twp, int tid) {
  c32 v[PS::ROUNDS][PS::R];
  lds_load<PS, B, T>(buf, v, tid);
  if constexpr (!PS::in_place) __syncthreads();
#pragma unroll
  for (int r = 0; r < PS::ROUNDS; ++r) {
    const int g = tid + r * T;
    if (PS::full() || g < PS::TOT) PS::template butterfly_own<INV>(v[r], g / B, twp);
  }
  lds_store<PS, B, T>(buf, v, tid);
  __syncthreads();
}

// Host: forward twiddles of every pass of a Stockham plan, packed as [pass][k][q-1] =
// W_{Ns r}^{k q}, computed in double precision and rounded once to float.
template <class RS>
std::vector<c32> host_stockham_twiddles() {
  std::vector<c32> t(tw_size<RS>() > 0 ? tw_size<RS>() : 1, c32{1.f, 0.f});
  int off = 0, ns = 1;
  for (int p = 0; p < RS::count; ++p) {
    const int R = RS::values[p];
    const int span = ns * R;
    for (int k = 0; k < ns; ++k)
      for (int q = 1; q < R; ++q) {
        const long m = (long)k * q % span;
        const double a = -2.0 * 3.14159265358979323846 * (double)m / (double)span;
        t[off + k * (R - 1) + (q - 1)] = c32{(float)std::cos(a), (float)std::sin(a)};
      }
    off += ns * (R - 1);
    ns *= R;
  }
  return t;
}

template <class RS>
std::vector<c32> host_twiddles() {
  if constexpr (RS::pfa) {
    return std::vector<c32>(1, c32{1.f, 0.f});  // prime-factor plans take no twiddles
  } else {
    return host_stockham_twiddles<RS>();
  }
}

// Host twiddle table of plan kind k for length L: the number of entries, of which at
// most cap are written to out (out may be null); -1 if the plan does not exist.
inline int twiddle_table(int kind, int L, c32* out, int cap) {
  std::vector<c32> t;
  switch (kind) {
    case kRowPlan:
      switch (L) {
#define PRNU_TW_ROW(X) \
  case X: t = host_twiddles<typename RowPlan<X>::RS>(); break;
        PRNU_FOR_EACH_LENGTH(PRNU_TW_ROW)
#undef PRNU_TW_ROW
        default: return -1;
      }
      break;
    case kColPlan:
    case kColPlanRev:
      switch (L) {
#define PRNU_TW_COL(X)                                                \
  case X:                                                             \
    t = kind == kColPlan ? host_twiddles<typename ColPlan<X>::RS>()    \
                         : host_twiddles<Reverse<typename ColPlan<X>::RS>>(); \
    break;
        PRNU_FOR_EACH_COL_LENGTH(PRNU_TW_COL)
#undef PRNU_TW_COL
        default: return -1;
      }
      break;
    default: return -1;
  }
  for (int i = 0; out && i < (int)t.size() && i < cap; ++i) out[i] = t[i];
  return (int)t.size();
}

}  // namespace prnu
