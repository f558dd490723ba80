// Noise residuals W(I) = I - F(I) (Sec. 2, before Eq. (2)) with the wavelet denoiser
// the paper cites, on the device.
//
//   k_dwt_fwd   one level of the periodic orthonormal 2-D wavelet transform with the
//               8-tap Daubechies filter: an LDS tile of the input (with the filter's
//               reach), the horizontal lowpass/highpass at even offsets, then the
//               vertical ones; the approximation goes to a plane of its own, the three
//               detail subbands to their quadrants of the coefficient plane.  Level 1
//               reads the caller's image and extends it by mirroring past its last row
//               and column (to a multiple of 16 on each side).
//   k_wiener    per detail subband: the windowed means of c^2 over 3x3, 5x5, 7x7 and
//               9x9 (zero outside the subband, separable sums in LDS), the smallest
//               minus s0^2 clipped at zero as the signal variance v, and the part the
//               Wiener estimate removes, c s0^2 / (v + s0^2).
//   k_dwt_inv   one level of the inverse transform (the adjoint, periodic) from the
//               approximation (zero at the coarsest level: the residual keeps none of
//               it) and the Wiener-removed detail parts; level 1 writes the cropped
//               residual.
//
// All arithmetic is fp32.  Every kernel is a streaming pass: its input tile and halo
// are read once into LDS, its outputs written once.
#include "kernels.hpp"

namespace prnu {

namespace {

// Daubechies' orthonormal 8-tap lowpass filter (4 vanishing moments, minimum phase),
// sum sqrt(2); the highpass is its quadrature mirror g[k] = (-1)^k h[7 - k].
__constant__ float kH[8] = {0.2303778133088964f,  0.7148465705529154f,  0.6308807679298587f,
                            -0.0279837694168599f, -0.1870348117190931f, 0.0308413818355607f,
                            0.0328830116668852f,  -0.0105974017850690f};
__constant__ float kG[8] = {-0.0105974017850690f, -0.0328830116668852f, 0.0308413818355607f,
                            0.1870348117190931f,  -0.0279837694168599f, -0.6308807679298587f,
                            0.7148465705529154f,  -0.2303778133088964f};

__device__ __forceinline__ int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// ---------------------------------------------------------------------------
// Forward level.  Output tile: FY rows x FX columns of each subband.

constexpr int FY = 16, FX = 32, FT = 256;
constexpr int FIY = 2 * FY + 6, FIX = 2 * FX + 6;  // input tile with the filter's reach

// in: level input plane of rows x cols (row stride in_rs, image stride in_is); at level 1
// the caller's M x N image, extended by mirroring to rows x cols.  ll: approximation
// plane (rows/2 x cols/2, stride ll_rs, image stride ll_is) or null.  det: coefficient
// plane of the image (stride det_rs, image stride det_is); the level's details go to its
// quadrants: (0, cols/2) horizontal high, (rows/2, 0) vertical high, (rows/2, cols/2) both.
__global__ __launch_bounds__(FT) void k_dwt_fwd(const float* __restrict__ in, int64_t in_is, int64_t in_rs, int rows,
                                                int cols, int M, int N, float* __restrict__ ll, int64_t ll_is,
                                                int64_t ll_rs, float* __restrict__ det, int64_t det_is,
                                                int64_t det_rs) {
  __shared__ float tile[FIY][FIX + 1];
  __shared__ float lo[FIY][FX + 1], hi[FIY][FX + 1];
  const int img = blockIdx.z;
  const int n0 = blockIdx.y * FY, m0 = blockIdx.x * FX;
  const float* src = in + (int64_t)img * in_is;
  for (int i = threadIdx.x; i < FIY * FIX; i += FT) {
    const int r = i / FIX, c = i % FIX;
    int y = wrap(2 * n0 + r, rows), x = wrap(2 * m0 + c, cols);
    if (y >= M) y = 2 * (M - 1) - y;  // mirror past the last row (level 1 only)
    if (x >= N) x = 2 * (N - 1) - x;
    tile[r][c] = src[(int64_t)y * in_rs + x];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < FIY * FX; i += FT) {
    const int r = i / FX, m = i % FX;
    float a = 0.f, b = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float v = tile[r][2 * m + k];
      a = fmaf(kH[k], v, a);
      b = fmaf(kG[k], v, b);
    }
    lo[r][m] = a;
    hi[r][m] = b;
  }
  __syncthreads();
  const int ro = rows / 2, co = cols / 2;
  float* d = det + (int64_t)img * det_is;
  for (int i = threadIdx.x; i < FY * FX; i += FT) {
    const int n = i / FX, m = i % FX;
    const int yo = n0 + n, xo = m0 + m;
    if (yo >= ro || xo >= co) continue;
    float s_ll = 0.f, s_lh = 0.f, s_hl = 0.f, s_hh = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float l = lo[2 * n + k][m], h = hi[2 * n + k][m];
      s_ll = fmaf(kH[k], l, s_ll);
      s_lh = fmaf(kG[k], l, s_lh);
      s_hl = fmaf(kH[k], h, s_hl);
      s_hh = fmaf(kG[k], h, s_hh);
    }
    if (ll) ll[(int64_t)img * ll_is + (int64_t)yo * ll_rs + xo] = s_ll;
    d[(int64_t)(yo + ro) * det_rs + xo] = s_lh;        // horizontal low, vertical high
    d[(int64_t)yo * det_rs + xo + co] = s_hl;          // horizontal high, vertical low
    d[(int64_t)(yo + ro) * det_rs + xo + co] = s_hh;
  }
}

// ---------------------------------------------------------------------------
// Wiener step on the detail subbands of one level.  Output tile WS x WS, halo 4.

constexpr int WS = 32, WH = 4, WT = 256, WE = WS + 2 * WH;

// coef / out: coefficient planes (stride rs, image stride is); the level's subbands
// are sr x sc at (0, sc), (sr, 0), (sr, sc).
__global__ __launch_bounds__(WT) void k_wiener(const float* __restrict__ coef, float* __restrict__ out, int64_t is,
                                               int64_t rs, int sr, int sc, float s2) {
  __shared__ float c2[WE][WE + 1];
  __shared__ float rsum[4][WE][WS + 1];
  const int img = blockIdx.z / 3, band = blockIdx.z % 3;
  const int oy = band == 0 ? 0 : sr, ox = band == 1 ? 0 : sc;
  const int y0 = blockIdx.y * WS, x0 = blockIdx.x * WS;
  const float* cb = coef + (int64_t)img * is + (int64_t)oy * rs + ox;
  float* ob = out + (int64_t)img * is + (int64_t)oy * rs + ox;
  for (int i = threadIdx.x; i < WE * WE; i += WT) {
    const int r = i / WE, c = i % WE;
    const int y = y0 + r - WH, x = x0 + c - WH;
    float v = 0.f;
    if (y >= 0 && y < sr && x >= 0 && x < sc) {
      v = cb[(int64_t)y * rs + x];
      v *= v;
    }
    c2[r][c] = v;
  }
  __syncthreads();
  // horizontal sums over 3, 5, 7, 9 columns centred on each interior column
  for (int i = threadIdx.x; i < WE * WS; i += WT) {
    const int r = i / WS, c = i % WS + WH;
    const float s3 = c2[r][c - 1] + c2[r][c] + c2[r][c + 1];
    const float s5 = s3 + c2[r][c - 2] + c2[r][c + 2];
    const float s7 = s5 + c2[r][c - 3] + c2[r][c + 3];
    const float s9 = s7 + c2[r][c - 4] + c2[r][c + 4];
    rsum[0][r][c - WH] = s3;
    rsum[1][r][c - WH] = s5;
    rsum[2][r][c - WH] = s7;
    rsum[3][r][c - WH] = s9;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < WS * WS; i += WT) {
    const int r = i / WS, c = i % WS;
    const int y = y0 + r, x = x0 + c;
    if (y >= sr || x >= sc) continue;
    const int R = r + WH;
    const float t3 = rsum[0][R - 1][c] + rsum[0][R][c] + rsum[0][R + 1][c];
    const float t5 = rsum[1][R - 2][c] + rsum[1][R - 1][c] + rsum[1][R][c] + rsum[1][R + 1][c] + rsum[1][R + 2][c];
    float t7 = 0.f, t9 = 0.f;
#pragma unroll
    for (int a = -3; a <= 3; ++a) t7 += rsum[2][R + a][c];
#pragma unroll
    for (int a = -4; a <= 4; ++a) t9 += rsum[3][R + a][c];
    const float m = fminf(fminf(t3 * (1.f / 9.f), t5 * (1.f / 25.f)), fminf(t7 * (1.f / 49.f), t9 * (1.f / 81.f)));
    const float v = fmaxf(0.f, m - s2);
    const float cv = cb[(int64_t)y * rs + x];
    ob[(int64_t)y * rs + x] = s2 > 0.f ? cv * (s2 / (v + s2)) : 0.f;
  }
}

// ---------------------------------------------------------------------------
// Inverse level.  Output tile IY x IX of the level's rows x cols plane.

constexpr int IY = 32, IX = 64, IT = 256;
constexpr int ICY = IY / 2 + 3, ICX = IX / 2 + 3;  // coefficient tile with the filter's reach

// ll: approximation plane (ro x co, stride ll_rs, image stride ll_is) or null (zero);
// det: detail parts, quadrants as in k_dwt_fwd.  out: rows x cols plane (stride out_rs,
// image stride out_is), only its first M rows and N columns written.
__global__ __launch_bounds__(IT) void k_dwt_inv(const float* __restrict__ ll, int64_t ll_is, int64_t ll_rs,
                                                const float* __restrict__ det, int64_t det_is, int64_t det_rs,
                                                int rows, int cols, int M, int N, float* __restrict__ out,
                                                int64_t out_is, int64_t out_rs) {
  __shared__ float s[4][ICY][ICX + 1];  // LL, LH, HL, HH
  __shared__ float vl[IY][ICX + 1], vh[IY][ICX + 1];
  const int img = blockIdx.z;
  const int ro = rows / 2, co = cols / 2;
  const int y0 = blockIdx.y * IY, x0 = blockIdx.x * IX;
  const int n0 = y0 / 2 - 3, m0 = x0 / 2 - 3;
  const float* d = det + (int64_t)img * det_is;
  const float* a = ll ? ll + (int64_t)img * ll_is : nullptr;
  for (int i = threadIdx.x; i < ICY * ICX; i += IT) {
    const int r = i / ICX, c = i % ICX;
    const int n = wrap(n0 + r, ro), m = wrap(m0 + c, co);
    s[0][r][c] = a ? a[(int64_t)n * ll_rs + m] : 0.f;
    s[1][r][c] = d[(int64_t)(n + ro) * det_rs + m];
    s[2][r][c] = d[(int64_t)n * det_rs + m + co];
    s[3][r][c] = d[(int64_t)(n + ro) * det_rs + m + co];
  }
  __syncthreads();
  // vertical: output row y takes coefficient rows y/2 - j (j = 0..3) with taps y%2 + 2j
  for (int i = threadIdx.x; i < IY * ICX; i += IT) {
    const int r = i / ICX, c = i % ICX;
    const int y = y0 + r, p = y & 1, nb = r / 2 + 3;
    float L = 0.f, H = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = p + 2 * j;
      L = fmaf(kH[k], s[0][nb - j][c], fmaf(kG[k], s[1][nb - j][c], L));
      H = fmaf(kH[k], s[2][nb - j][c], fmaf(kG[k], s[3][nb - j][c], H));
    }
    vl[r][c] = L;
    vh[r][c] = H;
  }
  __syncthreads();
  float* o = out + (int64_t)img * out_is;
  for (int i = threadIdx.x; i < IY * IX; i += IT) {
    const int r = i / IX, c = i % IX;
    const int y = y0 + r, x = x0 + c;
    if (y >= rows || x >= cols || y >= M || x >= N) continue;
    const int p = x & 1, mb = c / 2 + 3;
    float v = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = p + 2 * j;
      v = fmaf(kH[k], vl[r][mb - j], fmaf(kG[k], vh[r][mb - j], v));
    }
    o[(int64_t)y * out_rs + x] = v;
  }
}

}  // namespace

int residual_padded(int n) { return (n + 15) / 16 * 16; }

size_t residual_workspace_floats(int M, int N) {
  const size_t M2 = (size_t)residual_padded(M), N2 = (size_t)residual_padded(N);
  return 2 * M2 * N2 + (M2 / 2) * (N2 / 2) + (M2 / 4) * (N2 / 4);
}

hipError_t launch_residuals(const float* in, int64_t in_is, int64_t in_rs, int L, int M, int N, float sigma0,
                            float* ws, float* out, int64_t out_is, int64_t out_rs, hipStream_t s) {
  if (L <= 0) return hipSuccess;
  const int M2 = residual_padded(M), N2 = residual_padded(N);
  const int64_t P = (int64_t)M2 * N2;
  const int64_t per = (int64_t)residual_workspace_floats(M, N);
  // per image: coefficient plane C, Wiener-part plane D, approximation planes T1, T2
  float* C = ws;
  float* D = ws + P;
  float* T1 = ws + 2 * P;
  float* T2 = T1 + (int64_t)(M2 / 2) * (N2 / 2);
  constexpr int kLevels = 4;
  // forward: level l reads a rows x cols plane and writes rows/2 x cols/2 subbands
  for (int l = 1; l <= kLevels; ++l) {
    const int rows = M2 >> (l - 1), cols = N2 >> (l - 1);
    const float* src;
    int64_t sis, srs;
    int mm, nn;
    if (l == 1) {
      src = in, sis = in_is, srs = in_rs, mm = M, nn = N;
    } else {
      src = (l % 2 == 0) ? T1 : T2;  // level l-1 wrote its approximation there
      sis = per, srs = cols, mm = rows, nn = cols;
    }
    float* dst_ll = l == kLevels ? nullptr : ((l % 2 == 1) ? T1 : T2);
    dim3 grid((unsigned)((cols / 2 + FX - 1) / FX), (unsigned)((rows / 2 + FY - 1) / FY), (unsigned)L);
    k_dwt_fwd<<<grid, FT, 0, s>>>(src, sis, srs, rows, cols, mm, nn, dst_ll, per, cols / 2, C, per, N2);
  }
  const float s2 = sigma0 * sigma0;
  for (int l = 1; l <= kLevels; ++l) {
    const int sr = M2 >> l, sc = N2 >> l;
    dim3 grid((unsigned)((sc + WS - 1) / WS), (unsigned)((sr + WS - 1) / WS), (unsigned)(3 * L));
    k_wiener<<<grid, WT, 0, s>>>(C, D, per, N2, sr, sc, s2);
  }
  // inverse: level l rebuilds the rows x cols plane from its rows/2 x cols/2 subbands.
  // Approximations: level 4 starts from zero and writes T2, level 3 reads T2 and writes
  // T1, level 2 reads T1 and writes the (free) top-left quadrant of C, level 1 reads it
  // and writes the cropped residual.
  for (int l = kLevels; l >= 1; --l) {
    const int rows = M2 >> (l - 1), cols = N2 >> (l - 1);
    const float* src_ll = nullptr;
    int64_t src_rs = 0;
    if (l == 3) src_ll = T2, src_rs = cols / 2;
    if (l == 2) src_ll = T1, src_rs = cols / 2;
    if (l == 1) src_ll = C, src_rs = N2;
    float* dst = out;
    int64_t dis = out_is, drs = out_rs;
    int mm = M, nn = N;
    if (l > 1) {
      dst = l == 4 ? T2 : (l == 3 ? T1 : C);
      dis = per, drs = l == 2 ? N2 : cols, mm = rows, nn = cols;
    }
    dim3 grid((unsigned)((cols + IX - 1) / IX), (unsigned)((rows + IY - 1) / IY), (unsigned)L);
    k_dwt_inv<<<grid, IT, 0, s>>>(src_ll, per, src_rs, D, per, N2, rows, cols, mm, nn, dst, dis, drs);
  }
  return hipGetLastError();
}

}  // namespace prnu
