// Host emulation of the device FFT passes: the same plans, index maps, butterflies
// and twiddle tables as the kernels, executed serially.  Built into a small test
// library so that transform logic can be checked without a GPU.
#include <cstring>
#include <vector>

#include "fft_exec.hpp"

namespace prnu {
namespace {

template <int L, int B, bool INV, int P = 0>
void emu_passes(c32* buf, const c32* tw) {
  using RS = typename PlanFor<L>::RS;
  if constexpr (P < RS::count) {
    constexpr int R = RS::values[P];
    constexpr int NS = span_before<RS>(P);
    using I = StockhamIdx<L, R, NS, B>;
    std::vector<c32> v((size_t)I::TOT * R);
    for (int g = 0; g < I::TOT; ++g) I::load(buf, g, &v[(size_t)g * R]);
    for (int g = 0; g < I::TOT; ++g)
      I::template compute_store<INV>(buf, g, &v[(size_t)g * R], tw + tw_offset<RS>(P));
    emu_passes<L, B, INV, P + 1>(buf, tw);
  }
}

template <int L, int B>
int emu_batch(int inverse, const float* in, float* out) {
  const std::vector<c32> tw = host_twiddles<L>();
  std::vector<c32> buf((size_t)lds_size<B>(L * B));
  // input layout [batch][L]; LDS layout interleaved [L][batch]
  for (int b = 0; b < B; ++b)
    for (int i = 0; i < L; ++i)
      buf[lds_slot<B>(i * B + b)] = c32{in[2 * ((size_t)b * L + i)], in[2 * ((size_t)b * L + i) + 1]};
  if (inverse)
    emu_passes<L, B, true>(buf.data(), tw.data());
  else
    emu_passes<L, B, false>(buf.data(), tw.data());
  for (int b = 0; b < B; ++b)
    for (int i = 0; i < L; ++i) {
      out[2 * ((size_t)b * L + i)] = buf[lds_slot<B>(i * B + b)].x;
      out[2 * ((size_t)b * L + i) + 1] = buf[lds_slot<B>(i * B + b)].y;
    }
  return 0;
}

template <int L>
int emu_run(int inverse, int batch, const float* in, float* out) {
  switch (batch) {
    case 1: return emu_batch<L, 1>(inverse, in, out);
    case 3: return emu_batch<L, 3>(inverse, in, out);
    case 8: return emu_batch<L, 8>(inverse, in, out);
    default: return -1;
  }
}

}  // namespace
}  // namespace prnu

extern "C" int prnu_emu_fft(int length, int inverse, int batch, const float* in, float* out) {
  switch (length) {
#define PRNU_EMU_CASE(L) \
  case L: return prnu::emu_run<L>(inverse, batch, in, out);
    PRNU_FOR_EACH_LENGTH(PRNU_EMU_CASE)
#undef PRNU_EMU_CASE
    default: return -2;
  }
}

extern "C" int prnu_emu_lengths(int* out, int cap) {
  int n = 0;
#define PRNU_EMU_LEN(L) \
  if (n < cap) out[n] = L; \
  ++n;
  PRNU_FOR_EACH_LENGTH(PRNU_EMU_LEN)
#undef PRNU_EMU_LEN
  return n;
}
