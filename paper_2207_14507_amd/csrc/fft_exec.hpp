// Pass sequencing for the Stockham building blocks: the device version (LDS +
// workgroup barriers) and the host twiddle tables.
#pragma once

#include <cmath>
#include <vector>

#include "fft_plans.hpp"

namespace prnu {

// Run every pass of the plan for length L on B interleaved transforms in LDS with T
// threads.  The caller must have made the data visible (barrier) before the call; the
// data is visible to all threads on return.
template <int L, int B, int T, bool INV, int P = 0>
__device__ __forceinline__ void fft_lds(c32* buf, const c32* __restrict__ tw, int tid) {
  using RS = typename PlanFor<L>::RS;
  if constexpr (P < RS::count) {
    constexpr int R = RS::values[P];
    constexpr int NS = span_before<RS>(P);
    using I = StockhamIdx<L, R, NS, B>;
    constexpr int ROUNDS = (I::TOT + T - 1) / T;
    c32 v[ROUNDS][R];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
      const int g = tid + r * T;
      if (I::TOT % T == 0 || g < I::TOT) I::load(buf, g, v[r]);
    }
    __syncthreads();
    const c32* twp = tw + tw_offset<RS>(P);
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
      const int g = tid + r * T;
      if (I::TOT % T == 0 || g < I::TOT) I::template compute_store<INV>(buf, g, v[r], twp);
    }
    __syncthreads();
    fft_lds<L, B, T, INV, P + 1>(buf, tw, tid);
  }
}

// Host: forward twiddles of every pass, packed as [pass][k][q-1] = W_{Ns r}^{k q},
// computed in double precision and rounded once to float.
template <int L>
std::vector<c32> host_twiddles() {
  using RS = typename PlanFor<L>::RS;
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

}  // namespace prnu
