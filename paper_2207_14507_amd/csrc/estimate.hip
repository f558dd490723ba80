// Eq. (2) on the device: the reference fingerprint from L images and their noise
// residuals.
#include "kernels.hpp"

namespace prnu {

namespace {

// Eq. (2): reference fingerprint K = sum_l I_l W_l / sum_l I_l^2, pixel-wise, with FP64
// accumulators.  Each thread owns four consecutive pixels (16-byte loads when M N is a
// multiple of 4, the buffers being 16-byte aligned) and streams the L images and
// residuals once; zero where the images are dark.

template <int T>
__global__ __launch_bounds__(T) void k_estimate_fp(const float* __restrict__ I, const float* __restrict__ W,
                                                   int L, int64_t MN, float* __restrict__ K) {
  const int64_t p0 = ((int64_t)blockIdx.x * T + threadIdx.x) * 4;
  if (p0 >= MN) return;
  double n[4] = {0.0, 0.0, 0.0, 0.0}, d[4] = {0.0, 0.0, 0.0, 0.0};
  if ((MN & 3) == 0) {  // then p0 + 4 <= MN and every image row of four is 16-byte aligned
#pragma unroll 4
    for (int l = 0; l < L; ++l) {
      const float4 i = *reinterpret_cast<const float4*>(I + (int64_t)l * MN + p0);
      const float4 w = *reinterpret_cast<const float4*>(W + (int64_t)l * MN + p0);
      n[0] = fma((double)i.x, (double)w.x, n[0]);
      n[1] = fma((double)i.y, (double)w.y, n[1]);
      n[2] = fma((double)i.z, (double)w.z, n[2]);
      n[3] = fma((double)i.w, (double)w.w, n[3]);
      d[0] = fma((double)i.x, (double)i.x, d[0]);
      d[1] = fma((double)i.y, (double)i.y, d[1]);
      d[2] = fma((double)i.z, (double)i.z, d[2]);
      d[3] = fma((double)i.w, (double)i.w, d[3]);
    }
    float4 k;
    k.x = d[0] > 0.0 ? (float)(n[0] / d[0]) : 0.f;
    k.y = d[1] > 0.0 ? (float)(n[1] / d[1]) : 0.f;
    k.z = d[2] > 0.0 ? (float)(n[2] / d[2]) : 0.f;
    k.w = d[3] > 0.0 ? (float)(n[3] / d[3]) : 0.f;
    *reinterpret_cast<float4*>(K + p0) = k;
  } else {
    for (int64_t p = p0; p < p0 + 4 && p < MN; ++p) {
      double nn = 0.0, dd = 0.0;
      for (int l = 0; l < L; ++l) {
        const double i = I[(int64_t)l * MN + p], w = W[(int64_t)l * MN + p];
        nn = fma(i, w, nn);
        dd = fma(i, i, dd);
      }
      K[p] = dd > 0.0 ? (float)(nn / dd) : 0.f;
    }
  }
}

}  // namespace

hipError_t launch_estimate_fp(const float* I, const float* W, int L, int64_t MN, float* K, hipStream_t s) {
  if (MN <= 0) return hipSuccess;
  const int64_t threads = (MN + 3) / 4;
  k_estimate_fp<256><<<dim3((unsigned)((threads + 255) / 256)), 256, 0, s>>>(I, W, L, MN, K);
  return hipGetLastError();
}

}  // namespace prnu
