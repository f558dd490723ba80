// Launch interface of the search kernels (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_device.hpp"

namespace prnu {

// One candidate of a batch: the inverse-warp coefficients a = cos(theta)/s,
// b = sin(theta)/s (sampling point B(q) = [[a, -b], [b, a]] (q - c) + c) and the frame
// it applies to.
struct CandParam {
  float a, b;
  int32_t frame;
  int32_t pad;
};

// Per-candidate result of the PCE kernel.
struct CandRecord {
  double pce;
  double rho;
  double peak;     // correlation value at the peak (Eq. 1 numerator, unnormalised)
  int32_t dx, dy;
};

struct Shape {
  int M, N, radius;
  __host__ __device__ int Nh() const { return N / 2; }
  __host__ __device__ int band_rows() const { return 2 * (radius + 5) + 1; }
  __host__ __device__ int row_pairs() const { return (M + 1) / 2; }
  __host__ __device__ int band_pairs() const { return (band_rows() + 1) / 2; }
};

// Column-strip width of the column pass.
constexpr int kColStrip = 8;
__host__ __device__ inline int col_strips(const Shape& s) { return (s.Nh() + kColStrip - 1) / kColStrip; }

struct Batch {
  Shape shape;
  int nc;                      // candidates in this batch
  const CandParam* cand;       // device [nc]
  // residual frames
  const void* frames;          // device, dtype-dependent
  int dtype;                   // 0 f32, 1 bf16
  const float* frame_scale;    // device [n_frames] (bf16)
  int64_t frame_stride, row_stride;
  // fingerprint
  const c32* FK;               // device [M][Nh] packed column spectrum
  double fp_norm;              // ||K - mean K||
  // workspace
  c32* inter;                  // [nc][M][Nh]
  c32* band;                   // [nc][band_rows][Nh]
  float* win;                  // [nc][band_rows][band_rows]
  double2* norm_part;          // [nc][row_pairs] (sum r, sum r^2)
  double* energy_part;         // [nc][col_strips]
  CandRecord* rec;             // [nc]
  const c32* twM;              // twiddles for length M
  const c32* twN;              // twiddles for length N
};

// Returns hipSuccess or the launch error.
hipError_t launch_warp_rowfft(const Batch& b, hipStream_t s);
hipError_t launch_col_product(const Batch& b, hipStream_t s);
hipError_t launch_band_rowifft(const Batch& b, hipStream_t s);
hipError_t launch_pce(const Batch& b, hipStream_t s);

// Fingerprint preparation: FP64 sums of K, K - mean, 2-D DFT into FK (packed).
// work: device scratch of at least M*N floats; inter: [M][Nh] complex scratch;
// sums: device double[M + 2]; stats_out: device double[2] (mean, norm).
hipError_t launch_fp_prepare(const float* K, int64_t row_stride, const Shape& sh, float* work,
                             c32* inter, double* sums, double* stats_out, c32* FK,
                             const c32* twM, const c32* twN, CandParam* ident, hipStream_t s);

bool length_supported(int L);      // as a row length (frame width)
bool col_length_supported(int L);  // as a column length (frame height)
int supported_lengths(int* out, int cap);
// Host-built twiddle table for length L (forward), count of complex values.
int twiddle_table(int L, c32* out, int cap);

}  // namespace prnu
