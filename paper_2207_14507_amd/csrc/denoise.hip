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

// i mod n in [0, n).  The tiles reach at most one period past either end except on the
// smallest levels, so the division is the rare path.
__device__ __forceinline__ int wrap(int i, int n) {
  if (i >= 0 && i < n) return i;
  if (i >= n && i < 2 * n) return i - n;
  if (i < 0 && i >= -n) return i + n;
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
  {
    // every load of the tile issued before the first LDS store
    constexpr int NL = (FIY * FIX + FT - 1) / FT;
    float v[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int i = threadIdx.x + k * FT;
      if (i < FIY * FIX) {
        const int r = i / FIX, c = i % FIX;
        int y = wrap(2 * n0 + r, rows), x = wrap(2 * m0 + c, cols);
        if (y >= M) y = 2 * (M - 1) - y;  // mirror past the last row (level 1 only)
        if (x >= N) x = 2 * (N - 1) - x;
        v[k] = src[(int64_t)y * in_rs + x];
      }
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int i = threadIdx.x + k * FT;
      if (i < FIY * FIX) tile[i / FIX][i % FIX] = v[k];
    }
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
// Wiener step on the detail subbands of one level.  Output tile WY rows x WX columns,
// halo 4 (the 9x9 window's reach).  A thread owns one column and WR consecutive rows:
// it forms the horizontal sums of c^2 of the WR + 8 rows it needs in registers (each
// coefficient read from LDS once per window offset) and slides the vertical sums
// down its rows, so a coefficient costs about 20 LDS reads instead of the 40 of a
// separate horizontal pass through LDS.

constexpr int WX = 64, WY = 32, WH = 4, WT = 256, WR = WY / (WT / WX);
constexpr int WEX = WX + 2 * WH, WEY = WY + 2 * WH;

// coef / out: coefficient planes (stride rs, image stride is); the level's subbands
// are sr x sc at (0, sc), (sr, 0), (sr, sc).
__global__ __launch_bounds__(WT) void k_wiener(const float* __restrict__ coef, float* __restrict__ out, int64_t is,
                                               int64_t rs, int sr, int sc, float s2) {
  __shared__ float cs[WEY][WEX + 1];  // coefficients of the tile and halo, zero outside the subband
  const int img = blockIdx.z / 3, band = blockIdx.z % 3;
  const int oy = band == 0 ? 0 : sr, ox = band == 1 ? 0 : sc;
  const int y0 = blockIdx.y * WY, x0 = blockIdx.x * WX;
  const float* cb = coef + (int64_t)img * is + (int64_t)oy * rs + ox;
  float* ob = out + (int64_t)img * is + (int64_t)oy * rs + ox;
  {
    constexpr int NL = (WEY * WEX + WT - 1) / WT;
    float v[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int i = threadIdx.x + k * WT;
      const int r = i / WEX, c = i % WEX;
      const int y = y0 + r - WH, x = x0 + c - WH;
      v[k] = (i < WEY * WEX && y >= 0 && y < sr && x >= 0 && x < sc) ? cb[(int64_t)y * rs + x] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int i = threadIdx.x + k * WT;
      if (i < WEY * WEX) cs[i / WEX][i % WEX] = v[k];
    }
  }
  __syncthreads();
  const int tx = threadIdx.x % WX, r0 = (threadIdx.x / WX) * WR;
  const int x = x0 + tx;
  if (x >= sc) return;
  // horizontal sums of c^2 over 3, 5, 7, 9 columns for tile rows r0 - 4 .. r0 + WR + 3
  float h3[WR + 8], h5[WR + 8], h7[WR + 8], h9[WR + 8];
#pragma unroll
  for (int k = 0; k < WR + 8; ++k) {
    float q[9];
#pragma unroll
    for (int b = 0; b < 9; ++b) {
      const float v = cs[r0 + k][tx + b];
      q[b] = v * v;
    }
    h3[k] = q[3] + q[4] + q[5];
    h5[k] = h3[k] + q[2] + q[6];
    h7[k] = h5[k] + q[1] + q[7];
    h9[k] = h7[k] + q[0] + q[8];
  }
#pragma unroll
  for (int j = 0; j < WR; ++j) {
    const int y = y0 + r0 + j;
    if (y < sr) {
      const int k = j + WH;  // this row's index in the h arrays
      const float t3 = h3[k - 1] + h3[k] + h3[k + 1];
      const float t5 = h5[k - 2] + h5[k - 1] + h5[k] + h5[k + 1] + h5[k + 2];
      float t7 = 0.f, t9 = 0.f;
#pragma unroll
      for (int a = -3; a <= 3; ++a) t7 += h7[k + a];
#pragma unroll
      for (int a = -4; a <= 4; ++a) t9 += h9[k + a];
      const float m = fminf(fminf(t3 * (1.f / 9.f), t5 * (1.f / 25.f)), fminf(t7 * (1.f / 49.f), t9 * (1.f / 81.f)));
      const float v = fmaxf(0.f, m - s2);
      const float c = cs[r0 + k][tx + WH];
      ob[(int64_t)y * rs + x] = s2 > 0.f ? c * (s2 / (v + s2)) : 0.f;
    }
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
  {
    constexpr int NL = (ICY * ICX + IT - 1) / IT;
    float v[NL][4];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int i = threadIdx.x + k * IT;
      if (i < ICY * ICX) {
        const int n = wrap(n0 + i / ICX, ro), m = wrap(m0 + i % ICX, co);
        v[k][0] = a ? a[(int64_t)n * ll_rs + m] : 0.f;
        v[k][1] = d[(int64_t)(n + ro) * det_rs + m];
        v[k][2] = d[(int64_t)n * det_rs + m + co];
        v[k][3] = d[(int64_t)(n + ro) * det_rs + m + co];
      }
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int i = threadIdx.x + k * IT;
      if (i < ICY * ICX) {
#pragma unroll
        for (int b = 0; b < 4; ++b) s[b][i / ICX][i % ICX] = v[k][b];
      }
    }
  }
  __syncthreads();
  // vertical: output row y takes coefficient rows y/2 - j (j = 0..3) with taps y%2 + 2j
  // (y0 is even).  A thread takes one coefficient column and 8 output rows, which
  // need 7 coefficient rows of each subband: read into registers once.
  static_assert(IY % 8 == 0 && (IY / 8) * ICX <= IT, "one vertical work item per thread");
  if (threadIdx.x < (IY / 8) * ICX) {
    const int c = threadIdx.x % ICX, g = threadIdx.x / ICX;
    float q[4][7];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int t = 0; t < 7; ++t) q[b][t] = s[b][4 * g + t][c];
#pragma unroll
    for (int rr = 0; rr < 8; ++rr) {
      const int p = rr & 1, nb = rr / 2 + 3;  // local coefficient row of j = 0, minus 4g
      float L = 0.f, H = 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = p + 2 * j;
        L = fmaf(kH[k], q[0][nb - j], fmaf(kG[k], q[1][nb - j], L));
        H = fmaf(kH[k], q[2][nb - j], fmaf(kG[k], q[3][nb - j], H));
      }
      vl[8 * g + rr][c] = L;
      vh[8 * g + rr][c] = H;
    }
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
    dim3 grid((unsigned)((sc + WX - 1) / WX), (unsigned)((sr + WY - 1) / WY), (unsigned)(3 * L));
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
