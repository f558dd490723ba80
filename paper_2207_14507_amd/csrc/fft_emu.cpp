// Host emulation of the device FFT passes: the same plans, index maps, butterflies
// and twiddle tables as the kernels, executed serially.  Built into a small test
// library so that transform logic can be checked without a GPU.
#include <cstring>
#include <vector>

#include "fft_exec.hpp"

namespace prnu {
namespace {

template <class RS, int B, bool INV, int P = 0>
void emu_passes(c32* buf, const c32* tw) {
  if constexpr (P < RS::count) {
    using PS = Pass<RS, P, B, 1>;
    std::vector<c32> v((size_t)PS::TOT * PS::R);
    for (int g = 0; g < PS::TOT; ++g)
      for (int q = 0; q < PS::R; ++q) v[(size_t)g * PS::R + q] = buf[lds_slot<B>(PS::in_el(g / B, q) * B + g % B)];
    for (int g = 0; g < PS::TOT; ++g) {
      c32* x = &v[(size_t)g * PS::R];
      PS::template butterfly<INV>(x, g / B, tw);
      for (int q = 0; q < PS::R; ++q) buf[lds_slot<B>(PS::out_el(g / B, q) * B + g % B)] = x[q];
    }
    emu_passes<RS, B, INV, P + 1>(buf, tw);
  }
}

template <class RS, int B>
int emu_batch(int inverse, const float* in, float* out) {
  constexpr int L = RS::product();
  const std::vector<c32> tw = host_twiddles<RS>();
  std::vector<c32> buf((size_t)lds_size<B>(L * B));
  // input layout [batch][L]; LDS layout interleaved [L][batch], element i of a
  // transform at the plan's position of input index i (the identity for Stockham
  // plans), output index i read back from the plan's output position
  for (int b = 0; b < B; ++b)
    for (int i = 0; i < L; ++i)
      buf[lds_slot<B>(RS::in_pos(i) * B + b)] = c32{in[2 * ((size_t)b * L + i)], in[2 * ((size_t)b * L + i) + 1]};
  if (inverse)
    emu_passes<RS, B, true>(buf.data(), tw.data());
  else
    emu_passes<RS, B, false>(buf.data(), tw.data());
  for (int b = 0; b < B; ++b)
    for (int i = 0; i < L; ++i) {
      out[2 * ((size_t)b * L + i)] = buf[lds_slot<B>(RS::out_pos(i) * B + b)].x;
      out[2 * ((size_t)b * L + i) + 1] = buf[lds_slot<B>(RS::out_pos(i) * B + b)].y;
    }
  return 0;
}

template <class RS>
int emu_run(int inverse, int batch, const float* in, float* out) {
  switch (batch) {
    case 1: return emu_batch<RS, 1>(inverse, in, out);
    case 3: return emu_batch<RS, 3>(inverse, in, out);
    case 4: return emu_batch<RS, 4>(inverse, in, out);
    case 8: return emu_batch<RS, 8>(inverse, in, out);
    default: return -1;
  }
}

}  // namespace
}  // namespace prnu

using namespace prnu;

// kind: 0 row plan, 1 column plan, 2 reversed column plan.
extern "C" int prnu_emu_fft(int kind, int length, int inverse, int batch, const float* in, float* out) {
  if (kind == kRowPlan) {
    switch (length) {
#define PRNU_EMU_ROW(L) \
  case L: return emu_run<typename RowPlan<L>::RS>(inverse, batch, in, out);
      PRNU_FOR_EACH_LENGTH(PRNU_EMU_ROW)
#undef PRNU_EMU_ROW
      default: return -2;
    }
  }
  switch (length) {
#define PRNU_EMU_COL(L)                                                                           \
  case L:                                                                                         \
    return kind == kColPlan ? emu_run<typename ColPlan<L>::RS>(inverse, batch, in, out)            \
                            : emu_run<Reverse<typename ColPlan<L>::RS>>(inverse, batch, in, out);
    PRNU_FOR_EACH_COL_LENGTH(PRNU_EMU_COL)
#undef PRNU_EMU_COL
    default: return -2;
  }
}

extern "C" int prnu_emu_lengths(int kind, int* out, int cap) {
  int n = 0;
#define PRNU_EMU_LEN(L) \
  if (n < cap) out[n] = L; \
  ++n;
  if (kind == kRowPlan) {
    PRNU_FOR_EACH_LENGTH(PRNU_EMU_LEN)
  } else {
    PRNU_FOR_EACH_COL_LENGTH(PRNU_EMU_LEN)
  }
#undef PRNU_EMU_LEN
  return n;
}
