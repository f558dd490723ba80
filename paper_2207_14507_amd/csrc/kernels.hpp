// Launch interface of the search kernels (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_device.hpp"

namespace prnu {

// One candidate of a batch: the inverse-warp coefficients a = cos(theta)/s,
// b = sin(theta)/s (sampling point B(q) = [[a, -b], [b, a]] (q - c) + c), the frame it
// applies to and the fingerprint it is scored against (slots of the batch's tables).
struct CandParam {
  float a, b;
  int32_t frame;
  int32_t fp;
};

// A frame slot: device base of one zero-bordered frame and, for bf16 storage, the
// device address of its scale.
struct FrameRef {
  const void* data;
  const float* scale;
};

// A fingerprint slot: packed column spectrum of K - mean and the norm of K - mean.
struct FpRef {
  const c32* FK;
  double norm;
};

// Per-candidate result of the PCE kernel.
struct CandRecord {
  double pce;
  double rho;
  double peak;     // correlation value at the peak (Eq. 1 numerator, unnormalised)
  int32_t dx, dy;
};

// M x N: transform size (the fingerprint's).  Frames of M x N, or smaller ones of
// (M - ey) x (N - ex), zero-padded: their rows and columns past the frame are zero, and
// the peak is sought over -R <= dy <= ey + R, -R <= dx <= ex + R (the linear shifts of
// Eq. (3) widened by the radius).  The stored window reaches 5 further on each side
// (the exclusion block): band_rows() x win_cols().
struct Shape {
  int M, N, radius;
  int ey = 0, ex = 0;
  __host__ __device__ int Nh() const { return N / 2; }
  __host__ __device__ int Mf() const { return M - ey; }
  __host__ __device__ int Nf() const { return N - ex; }
  __host__ __device__ bool padded() const { return (ey | ex) != 0; }
  __host__ __device__ int band_rows() const { return ey + 2 * (radius + 5) + 1; }
  __host__ __device__ int win_cols() const { return ex + 2 * (radius + 5) + 1; }
  __host__ __device__ int row_pairs() const { return (M + 1) / 2; }
  __host__ __device__ int band_pairs() const { return (band_rows() + 1) / 2; }
};

// Residual frames are staged with a zero border of kBorder pixels on every side, so that
// the bilinear taps of any sampling point clamped to [-1, N] x [-1, M] are in bounds and
// read zero outside the image, and as vertical pairs: entry (x, y) holds the bordered
// frame's pixels (x, y) and (x, y + 1), so that the four taps of a sampling point are
// one 16-byte load (8 bytes for bf16) at the entry of its top-left tap.  An M x N frame
// has padded_row(N) entries per row and pair_rows(M) rows of entries, 2 elements each.
constexpr int kBorder = 2;
__host__ __device__ constexpr inline int64_t padded_row(int N) { return N + 2 * kBorder; }
__host__ __device__ constexpr inline int64_t pair_rows(int M) { return M + 2 * kBorder - 1; }
// Elements (f32 or bf16 values) of one staged frame.
__host__ __device__ inline int64_t padded_frame(int M, int N) { return pair_rows(M) * padded_row(N) * 2; }

// Column-strip width of the column pass.
constexpr int kColStrip = 8;
__host__ __device__ inline int col_strips(const Shape& s) { return (s.Nh() + kColStrip - 1) / kColStrip; }
// Strip-tiled layout of a packed half spectrum of M rows (the row pass's output and the
// fingerprint spectrum): element (y, c) at (c / kColStrip) * M * kColStrip +
// y * kColStrip + c % kColStrip.  A column strip is one contiguous block, read whole by
// the column pass, and the two rows of a row pair are adjacent in it (128-byte runs for
// the row pass's stores).  Columns past N/2 in the last strip are padding.
__host__ __device__ inline int tiled_cols(const Shape& s) { return col_strips(s) * kColStrip; }
// Column workgroups per strip: a strip of 8 columns of 1280 rows or more would leave one
// workgroup per CU (its LDS, or its registers), so its two halves of 4 columns go to two
// workgroups.
__host__ __device__ constexpr inline int col_split(int M) { return M >= 1280 ? 2 : 1; }
// Column workgroups (and energy partial sums) per candidate.
__host__ __device__ inline int col_blocks(const Shape& s) { return col_strips(s) * col_split(s.M); }

struct Batch {
  Shape shape;
  int nc;                      // candidates in this batch
  const CandParam* cand;       // device [nc]
  // residual frames of shape.Mf() x shape.Nf(), staged zero-bordered as vertical pairs
  // (entry (x, y) = bordered pixels (x, y) and (x, y + 1); padded_row(Nf) entries per
  // row, the image pixel (y, x) at bordered (y + kBorder, x + kBorder)), all of one
  // dtype: 0 f32, 1 bf16
  int dtype;
  const FrameRef* frames;      // device, indexed by CandParam::frame
  const FpRef* fps;            // device, indexed by CandParam::fp
  // workspace
  c32* inter;                  // [nc] x strip-tiled M x tiled_cols
  c32* band;                   // [nc][band_rows][Nh]
  float* win;                  // [nc][band_rows][win_cols]
  double2* norm_part;          // [nc][row_pairs] (sum r, sum r^2)
  double* energy_part;         // [nc][col_blocks]
  CandRecord* rec;             // [nc]
  const c32* twM;              // twiddles of the column plan (length M)
  const c32* twMi;             // twiddles of the reversed column plan
  const c32* twN;              // twiddles of the row plan (length N)
  // Block-to-work order of the row and column kernels: 0 = candidate fastest (blocks
  // next in line share a row pair or column strip, so the frame rows and fingerprint
  // strip are reused from cache), 1 = tile fastest (a candidate's tiles run together).
  int order;
  // General Eq. (4) candidates: per candidate (indexed like cand), the 9 entries of
  // G = T^-1 (row-major, centred coordinates); the row kernel then samples at
  // (G00 ux + G01 uy + G02, G10 ux + G11 uy + G12) / (G20 ux + G21 uy + G22) + c.  Null
  // for the similarity form (CandParam::a, b).
  const float* proj;
  // Device-counted launch (null: nc candidates): this batch is the chunk starting at
  // list position dyn_start of a candidate list whose length the device writes to
  // *nc_dev before the launch runs; it processes min(nc, *nc_dev - dyn_start) candidates
  // (none when that is not positive) with a fixed grid that strides over the tiles.
  // Similarity candidates only (proj must be null).
  const int* nc_dev;
  int dyn_start;
  // Launch shape of a device-counted launch (the kernels do not read it): 1 = one
  // workgroup per tile of the whole chunk (fastest when the chunk holds work; an empty
  // one still dispatches every workgroup), 0 = a grid of a few workgroups per CU
  // striding over the tiles (cheap when empty, slower per tile).
  int dyn_full;
};

// Returns hipSuccess or the launch error.
hipError_t launch_warp_rowfft(const Batch& b, hipStream_t s);
hipError_t launch_col_product(const Batch& b, hipStream_t s);
hipError_t launch_band_rowifft(const Batch& b, hipStream_t s);
hipError_t launch_pce(const Batch& b, hipStream_t s);

// Copy n frames (element size 4 = f32 or 2 = bf16 bits) into the staged layout (zero
// border, vertical pairs).
hipError_t launch_pad_frames(const void* src, int elem_bytes, int64_t src_frame_stride, int64_t src_row_stride,
                             int n_frames, int M, int N, void* dst, hipStream_t s);

// Eq. (2) over L tight M x N fp32 images and residuals (16-byte aligned) into K
// (estimate.hip).
hipError_t launch_estimate_fp(const float* I, const float* W, int L, int64_t MN, float* K, hipStream_t s);

// Noise residuals W(I) = I - F(I) of L fp32 images of M x N (M, N >= 9; image and row
// strides in elements) into out (image and row strides in elements), with the wavelet
// denoiser at noise standard deviation sigma0 (denoise.hip).  ws: device workspace of
// L * residual_workspace_floats(M, N) floats.
size_t residual_workspace_floats(int M, int N);
hipError_t launch_residuals(const float* in, int64_t in_is, int64_t in_rs, int L, int M, int N, float sigma0,
                            float* ws, float* out, int64_t out_is, int64_t out_rs, hipStream_t s);

// Fingerprint preparation: FP64 sums of K, K - mean, 2-D DFT into FK (packed).
// work: device scratch of at least padded_frame(M, N) floats (K - mean in the staged
// layout); inter: [M][Nh] complex scratch;
// sums: device double[M + 2]; stats_out: device double[2] (mean, norm); ident: device
// candidate {1, 0, 0, 0}; wref: device FrameRef {work, null}.
hipError_t launch_fp_prepare(const float* K, int64_t row_stride, const Shape& sh, float* work,
                             c32* inter, double* sums, double* stats_out, c32* FK,
                             const c32* twM, const c32* twMi, const c32* twN, const CandParam* ident,
                             const FrameRef* wref, hipStream_t s);

bool length_supported(int L);      // as a row length (frame width)
bool col_length_supported(int L);  // as a column length (frame height)
int supported_lengths(int* out, int cap);

}  // namespace prnu
