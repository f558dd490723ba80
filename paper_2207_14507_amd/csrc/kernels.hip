// Search kernels for gfx950: per batch of candidates, the correlation surface of
// Eq. (1) near zero shift and the PCE of Eq. (3).
//
//   k_warp_rowfft   inverse warp of the residual (Eq. 4, similarity form, bilinear,
//                   zero outside) fused with the row DFT: two warped rows form one
//                   complex row, transformed in LDS and split into the two half
//                   spectra.  Packed half-spectrum layout per row: slot 0 holds the
//                   two real bins (DC, Nyquist), slots 1..N/2-1 the complex bins.
//                   Also FP64 sums of the warped values (norm of Eq. 1).
//   k_col_product   column DFT of a strip of the packed half spectrum, product with
//                   the conjugated residual spectrum, FP64 Parseval energy of the
//                   product (all-shift energy of Eq. 3), inverse column DFT; only the
//                   rows |dy| <= R + 5 (peak search + exclusion reach) are stored.
//   k_band_rowifft  inverse row DFT of pairs of stored rows (Hermitian-extended);
//                   only the columns |dx| <= R + 5 are stored.
//   k_pce           signed peak over |dy|,|dx| <= R, FP64 energy of the 11x11
//                   exclusion block, PCE and NCC at the peak.
//
// All transforms are unnormalised; the 1/(MN) factors are applied in FP64 in k_pce.
#include <math.h>

#include "fft_exec.hpp"
#include "kernels.hpp"

namespace prnu {

namespace {

template <int T>
__device__ inline double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  constexpr int W = (T + 63) / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < W; ++i) s += red[i];
  }
  return s;  // valid in thread 0
}

template <int DT>
__device__ __forceinline__ float fetch(const char* base, int64_t idx, float scale) {
  if constexpr (DT == 0) {
    return reinterpret_cast<const float*>(base)[idx];
  } else {
    const unsigned short h = reinterpret_cast<const unsigned short*>(base)[idx];
    return __uint_as_float((unsigned)h << 16) * scale;
  }
}

// Bilinear sample of the residual at B(q) = [[a, -b], [b, a]] (q - c) + c, q - c = (ux, uy).
// Taps outside the M x N image contribute zero and are never read.
template <int DT>
__device__ __forceinline__ float sample(const char* base, int64_t rs, int M, int N, float a, float b,
                                        float ux, float uy, float cx, float cy, float scale) {
  const float xs = fmaf(a, ux, fmaf(-b, uy, cx));
  const float ys = fmaf(b, ux, fmaf(a, uy, cy));
  const float xf = floorf(xs), yf = floorf(ys);
  const float fx = xs - xf, fy = ys - yf;
  const int x0 = (int)xf, y0 = (int)yf;
  const bool vx0 = (unsigned)x0 < (unsigned)N, vx1 = (unsigned)(x0 + 1) < (unsigned)N;
  const bool vy0 = (unsigned)y0 < (unsigned)M, vy1 = (unsigned)(y0 + 1) < (unsigned)M;
  const int64_t r0 = (int64_t)y0 * rs, r1 = r0 + rs;
  const float w00 = (vy0 && vx0) ? fetch<DT>(base, r0 + x0, scale) : 0.f;
  const float w01 = (vy0 && vx1) ? fetch<DT>(base, r0 + x0 + 1, scale) : 0.f;
  const float w10 = (vy1 && vx0) ? fetch<DT>(base, r1 + x0, scale) : 0.f;
  const float w11 = (vy1 && vx1) ? fetch<DT>(base, r1 + x0 + 1, scale) : 0.f;
  const float top = fmaf(fx, w01 - w00, w00);
  const float bot = fmaf(fx, w11 - w10, w10);
  return fmaf(fy, bot - top, top);
}

// ---------------------------------------------------------------------------

template <int N, int T, int DT>
__global__ __launch_bounds__(T) void k_warp_rowfft(Batch bt) {
  __shared__ c32 buf[N];
  __shared__ double red[(T + 63) / 64];
  const int nc = bt.nc;
  const int ci = blockIdx.x % nc;
  const int pair = blockIdx.x / nc;
  const int M = bt.shape.M;
  const CandParam cp = bt.cand[ci];
  const int y0 = 2 * pair, y1 = y0 + 1;
  const bool has1 = y1 < M;
  const float cx = 0.5f * (float)(N - 1), cy = 0.5f * (float)(M - 1);
  const float scale = (DT == 1) ? bt.frame_scale[cp.frame] : 1.f;
  const char* base = reinterpret_cast<const char*>(bt.frames) +
                     (size_t)cp.frame * (size_t)bt.frame_stride * (DT == 1 ? 2 : 4);
  const float uy0 = (float)y0 - cy, uy1 = (float)y1 - cy;
  double s1 = 0.0, s2 = 0.0;
  for (int x = threadIdx.x; x < N; x += T) {
    const float ux = (float)x - cx;
    const float r0 = sample<DT>(base, bt.row_stride, M, N, cp.a, cp.b, ux, uy0, cx, cy, scale);
    const float r1 = has1 ? sample<DT>(base, bt.row_stride, M, N, cp.a, cp.b, ux, uy1, cx, cy, scale) : 0.f;
    buf[x] = c32{r0, r1};
    s1 += (double)r0 + (double)r1;
    s2 = fma((double)r0, (double)r0, fma((double)r1, (double)r1, s2));
  }
  __syncthreads();
  fft_lds<N, 1, T, false>(buf, bt.twN, threadIdx.x);
  constexpr int Nh = N / 2;
  c32* o0 = bt.inter + ((size_t)ci * M + y0) * Nh;
  c32* o1 = o0 + Nh;
  for (int k = threadIdx.x; k < Nh; k += T) {
    const c32 z = buf[k];
    c32 x0, x1;
    if (k == 0) {
      const c32 zh = buf[Nh];
      x0 = c32{z.x, zh.x};
      x1 = c32{z.y, zh.y};
    } else {
      const c32 zm = buf[N - k];
      x0 = c32{0.5f * (z.x + zm.x), 0.5f * (z.y - zm.y)};
      x1 = c32{0.5f * (z.y + zm.y), -0.5f * (z.x - zm.x)};
    }
    o0[k] = x0;
    if (has1) o1[k] = x1;
  }
  s1 = block_sum<T>(s1, red);
  s2 = block_sum<T>(s2, red);
  if (threadIdx.x == 0) bt.norm_part[(size_t)ci * bt.shape.row_pairs() + pair] = make_double2(s1, s2);
}

// ---------------------------------------------------------------------------

template <int M, int T, bool PRODUCT>
__global__ __launch_bounds__(T) void k_col(Batch bt, c32* fk_out) {
  constexpr int CW = kColStrip;
  __shared__ c32 buf[M * CW];
  __shared__ double red[(T + 63) / 64];
  const int nc = bt.nc;
  const int ci = blockIdx.x % nc;
  const int strip = blockIdx.x / nc;
  const int Nh = bt.shape.N / 2;
  const int col0 = strip * CW;
  const c32* src = bt.inter + (size_t)ci * M * Nh;
  for (int idx = threadIdx.x; idx < M * CW; idx += T) {
    const int row = idx / CW, c = idx % CW, col = col0 + c;
    buf[idx] = col < Nh ? src[(size_t)row * Nh + col] : c32{0.f, 0.f};
  }
  __syncthreads();
  fft_lds<M, CW, T, false>(buf, bt.twM, threadIdx.x);
  if constexpr (!PRODUCT) {
    for (int idx = threadIdx.x; idx < M * CW; idx += T) {
      const int row = idx / CW, c = idx % CW, col = col0 + c;
      if (col >= Nh) continue;
      c32 v = buf[idx];
      if (row == 0 && col == 0) v.x = 0.f;  // DC of the mean-free fingerprint is exactly zero
      fk_out[(size_t)row * Nh + col] = v;
    }
  } else {
    const c32* FK = bt.FK;
    double e = 0.0;
    for (int idx = threadIdx.x; idx < M * CW; idx += T) {
      const int row = idx / CW, c = idx % CW, col = col0 + c;
      if (col >= Nh || col == 0) continue;
      const c32 g = cmulc(FK[(size_t)row * Nh + col], buf[idx]);
      e = fma(2.0 * (double)g.x, (double)g.x, fma(2.0 * (double)g.y, (double)g.y, e));
      buf[idx] = g;
    }
    if (col0 == 0) {
      // Slot 0 packs two real columns (x-bins 0 and N/2): split each spectrum by
      // Hermitian symmetry in ky, multiply, and pack the two products again.
      for (int ky = threadIdx.x; ky <= M / 2; ky += T) {
        const int kn = (M - ky) % M;
        const c32 z = buf[ky * CW], zn = buf[kn * CW];
        const c32 zk = FK[(size_t)ky * Nh], zkn = FK[(size_t)kn * Nh];
        const c32 A = {0.5f * (z.x + zn.x), 0.5f * (z.y - zn.y)};
        const c32 B = {0.5f * (z.y + zn.y), -0.5f * (z.x - zn.x)};
        const c32 FA = {0.5f * (zk.x + zkn.x), 0.5f * (zk.y - zkn.y)};
        const c32 FB = {0.5f * (zk.y + zkn.y), -0.5f * (zk.x - zkn.x)};
        const c32 GA = cmulc(FA, A), GB = cmulc(FB, B);
        const double eg = (double)GA.x * GA.x + (double)GA.y * GA.y + (double)GB.x * GB.x + (double)GB.y * GB.y;
        buf[ky * CW] = c32{GA.x - GB.y, GA.y + GB.x};
        if (kn != ky) {
          buf[kn * CW] = c32{GA.x + GB.y, GB.x - GA.y};
          e += 2.0 * eg;
        } else {
          e += eg;
        }
      }
    }
    __syncthreads();
    fft_lds<M, CW, T, true>(buf, bt.twM, threadIdx.x);
    const int H = bt.shape.radius + 5, BR = 2 * H + 1;
    c32* dst = bt.band + (size_t)ci * BR * Nh;
    for (int idx = threadIdx.x; idx < BR * CW; idx += T) {
      const int br = idx / CW, c = idx % CW, col = col0 + c;
      if (col >= Nh) continue;
      int srow = br - H;
      srow += (srow < 0) ? M : 0;
      dst[(size_t)br * Nh + col] = buf[srow * CW + c];
    }
    e = block_sum<T>(e, red);
    if (threadIdx.x == 0) bt.energy_part[(size_t)ci * col_strips(bt.shape) + strip] = e;
  }
}

// ---------------------------------------------------------------------------

template <int N, int T>
__global__ __launch_bounds__(T) void k_band_rowifft(Batch bt) {
  __shared__ c32 buf[N];
  constexpr int Nh = N / 2;
  const int nc = bt.nc;
  const int ci = blockIdx.x % nc;
  const int p = blockIdx.x / nc;
  const int H = bt.shape.radius + 5, BR = 2 * H + 1;
  const int ra = 2 * p, rb = ra + 1;
  const bool hasb = rb < BR;
  const c32* ba = bt.band + ((size_t)ci * BR + ra) * Nh;
  const c32* bb = ba + Nh;
  for (int kx = threadIdx.x; kx <= Nh; kx += T) {
    c32 ca, cb = {0.f, 0.f};
    if (kx == 0) {
      ca = c32{ba[0].x, 0.f};
      if (hasb) cb = c32{bb[0].x, 0.f};
    } else if (kx == Nh) {
      ca = c32{ba[0].y, 0.f};
      if (hasb) cb = c32{bb[0].y, 0.f};
    } else {
      ca = ba[kx];
      if (hasb) cb = bb[kx];
    }
    buf[kx] = c32{ca.x - cb.y, ca.y + cb.x};                       // ca + i cb
    if (kx != 0 && kx != Nh) buf[N - kx] = c32{ca.x + cb.y, cb.x - ca.y};  // conj(ca) + i conj(cb)
  }
  __syncthreads();
  fft_lds<N, 1, T, true>(buf, bt.twN, threadIdx.x);
  float* wa = bt.win + ((size_t)ci * BR + ra) * BR;
  float* wb = wa + BR;
  for (int i = threadIdx.x; i < BR; i += T) {
    int col = i - H;
    col += (col < 0) ? N : 0;
    const c32 z = buf[col];
    wa[i] = z.x;
    if (hasb) wb[i] = z.y;
  }
}

// ---------------------------------------------------------------------------

template <int T>
__global__ __launch_bounds__(T) void k_pce(Batch bt) {
  __shared__ double red[(T + 63) / 64];
  __shared__ float sbest[(T + 63) / 64];
  __shared__ int sidx[(T + 63) / 64];
  __shared__ int peak_idx;
  const int ci = blockIdx.x;
  const int R = bt.shape.radius, H = R + 5, BR = 2 * H + 1, S = 2 * R + 1;
  const float* w = bt.win + (size_t)ci * BR * BR;
  float best = -INFINITY;
  int bidx = 0x7fffffff;
  for (int idx = threadIdx.x; idx < S * S; idx += T) {
    const int r = idx / S, c = idx % S;
    const float v = w[(r + 5) * BR + (c + 5)];
    if (v > best) {
      best = v;
      bidx = idx;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const float ov = __shfl_xor(best, o, 64);
    const int oi = __shfl_xor(bidx, o, 64);
    if (ov > best || (ov == best && oi < bidx)) {
      best = ov;
      bidx = oi;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    sbest[wv] = best;
    sidx[wv] = bidx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (T + 63) / 64; ++i)
      if (sbest[i] > best || (sbest[i] == best && sidx[i] < bidx)) {
        best = sbest[i];
        bidx = sidx[i];
      }
    peak_idx = bidx;
    sbest[0] = best;
  }
  __syncthreads();
  const int pidx = peak_idx;
  const bool found = pidx != 0x7fffffff;
  const int pr = found ? pidx / S : R, pc = found ? pidx % S : R;
  // energy of the exclusion block (its centre is at window (pr + 5, pc + 5))
  double sd = 0.0;
  if (threadIdx.x < 121) {
    const int a = threadIdx.x / 11 - 5, b = threadIdx.x % 11 - 5;
    const double v = (double)w[(pr + 5 + a) * BR + (pc + 5 + b)];
    sd = v * v;
  }
  sd = block_sum<T>(sd, red);
  const int nstrips = col_strips(bt.shape);
  double e = 0.0;
  for (int i = threadIdx.x; i < nstrips; i += T) e += bt.energy_part[(size_t)ci * nstrips + i];
  e = block_sum<T>(e, red);
  const int np = bt.shape.row_pairs();
  double s1 = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < np; i += T) {
    const double2 v = bt.norm_part[(size_t)ci * np + i];
    s1 += v.x;
    s2 += v.y;
  }
  s1 = block_sum<T>(s1, red);
  s2 = block_sum<T>(s2, red);
  if (threadIdx.x == 0) {
    const double MN = (double)bt.shape.M * (double)bt.shape.N;
    const double cpk = (double)sbest[0] / MN;      // C at the peak
    const double all = e / MN;                     // sum over all shifts of C^2 (Parseval)
    const double excl = sd / (MN * MN);            // sum over the exclusion block
    const double off = all - excl;
    CandRecord r;
    r.pce = (found && off > 0.0) ? copysign(cpk * cpk, cpk) * (MN - 121.0) / off : (found ? 0.0 : NAN);
    const double rn2 = s2 - s1 * s1 / MN;
    r.rho = (rn2 > 0.0 && bt.fp_norm > 0.0) ? cpk / (bt.fp_norm * sqrt(rn2)) : 0.0;
    r.peak = cpk;
    r.dx = pc - R;
    r.dy = pr - R;
    bt.rec[ci] = r;
  }
}

// ---------------------------------------------------------------------------
// Fingerprint preparation.

template <int T>
__global__ __launch_bounds__(T) void k_fp_rowsums(const float* K, int64_t rs, int M, int N, const double* mean,
                                                  double* part) {
  __shared__ double red[(T + 63) / 64];
  const int y = blockIdx.x;
  const double mu = mean ? *mean : 0.0;
  double s = 0.0;
  for (int x = threadIdx.x; x < N; x += T) {
    const double v = (double)K[(int64_t)y * rs + x] - mu;
    s += mean ? v * v : v;
  }
  s = block_sum<T>(s, red);
  if (threadIdx.x == 0) part[y] = s;
}

template <int T>
__global__ __launch_bounds__(T) void k_fp_finish(const double* part, int M, double count, double* out, int second) {
  __shared__ double red[(T + 63) / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < M; i += T) s += part[i];
  s = block_sum<T>(s, red);
  if (threadIdx.x == 0) {
    if (!second) out[0] = s / count;  // mean
    else out[1] = sqrt(s);            // norm of K - mean
  }
}

template <int T>
__global__ __launch_bounds__(T) void k_fp_center(const float* K, int64_t rs, int M, int N, const double* mean,
                                                 float* out) {
  const int y = blockIdx.x;
  const double mu = *mean;
  for (int x = threadIdx.x; x < N; x += T) out[(int64_t)y * N + x] = (float)((double)K[(int64_t)y * rs + x] - mu);
}

// ---------------------------------------------------------------------------
// Dispatch.

template <int N>
constexpr int row_threads() {
  return N >= 3840 ? 128 : 64;
}
template <int M>
constexpr int col_threads() {
  return M >= 2160 ? 512 : 256;
}

template <int N>
hipError_t launch_rows(const Batch& b, hipStream_t s) {
  constexpr int T = row_threads<N>();
  dim3 grid((unsigned)(b.nc * b.shape.row_pairs()));
  if (b.dtype == 1)
    k_warp_rowfft<N, T, 1><<<grid, T, 0, s>>>(b);
  else
    k_warp_rowfft<N, T, 0><<<grid, T, 0, s>>>(b);
  return hipGetLastError();
}

template <int M>
hipError_t launch_cols(const Batch& b, hipStream_t s, c32* fk_out) {
  constexpr int T = col_threads<M>();
  dim3 grid((unsigned)(b.nc * col_strips(b.shape)));
  if (fk_out)
    k_col<M, T, false><<<grid, T, 0, s>>>(b, fk_out);
  else
    k_col<M, T, true><<<grid, T, 0, s>>>(b, nullptr);
  return hipGetLastError();
}

template <int N>
hipError_t launch_band(const Batch& b, hipStream_t s) {
  constexpr int T = row_threads<N>();
  dim3 grid((unsigned)(b.nc * b.shape.band_pairs()));
  k_band_rowifft<N, T><<<grid, T, 0, s>>>(b);
  return hipGetLastError();
}

hipError_t dispatch_cols(const Batch& b, hipStream_t s, c32* fk_out) {
  switch (b.shape.M) {
#define PRNU_CASE(L) \
  case L: return launch_cols<L>(b, s, fk_out);
    PRNU_FOR_EACH_COL_LENGTH(PRNU_CASE)
#undef PRNU_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool length_supported(int L) {
  switch (L) {
#define PRNU_CASE(X) \
  case X: return true;
    PRNU_FOR_EACH_LENGTH(PRNU_CASE)
#undef PRNU_CASE
    default: return false;
  }
}

bool col_length_supported(int L) {
  switch (L) {
#define PRNU_CASE(X) \
  case X: return true;
    PRNU_FOR_EACH_COL_LENGTH(PRNU_CASE)
#undef PRNU_CASE
    default: return false;
  }
}

int supported_lengths(int* out, int cap) {
  int n = 0;
#define PRNU_CASE(X) \
  if (out && n < cap) out[n] = X; \
  ++n;
  PRNU_FOR_EACH_LENGTH(PRNU_CASE)
#undef PRNU_CASE
  return n;
}

int twiddle_table(int L, c32* out, int cap) {
  switch (L) {
#define PRNU_CASE(X)                                            \
  case X: {                                                     \
    const std::vector<c32> t = host_twiddles<X>();              \
    for (int i = 0; i < (int)t.size() && i < cap; ++i) out[i] = t[i]; \
    return (int)t.size();                                       \
  }
    PRNU_FOR_EACH_LENGTH(PRNU_CASE)
#undef PRNU_CASE
    default: return -1;
  }
}

hipError_t launch_warp_rowfft(const Batch& b, hipStream_t s) {
  switch (b.shape.N) {
#define PRNU_CASE(L) \
  case L: return launch_rows<L>(b, s);
    PRNU_FOR_EACH_LENGTH(PRNU_CASE)
#undef PRNU_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_col_product(const Batch& b, hipStream_t s) { return dispatch_cols(b, s, nullptr); }

hipError_t launch_band_rowifft(const Batch& b, hipStream_t s) {
  switch (b.shape.N) {
#define PRNU_CASE(L) \
  case L: return launch_band<L>(b, s);
    PRNU_FOR_EACH_LENGTH(PRNU_CASE)
#undef PRNU_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pce(const Batch& b, hipStream_t s) {
  k_pce<256><<<dim3((unsigned)b.nc), 256, 0, s>>>(b);
  return hipGetLastError();
}

hipError_t launch_fp_prepare(const float* K, int64_t row_stride, const Shape& sh, float* work, c32* inter,
                             double* sums, double* stats_out, c32* FK, const c32* twM, const c32* twN,
                             CandParam* ident, hipStream_t s) {
  const int M = sh.M, N = sh.N;
  k_fp_rowsums<256><<<M, 256, 0, s>>>(K, row_stride, M, N, nullptr, sums);
  k_fp_finish<256><<<1, 256, 0, s>>>(sums, M, (double)M * N, stats_out, 0);
  k_fp_rowsums<256><<<M, 256, 0, s>>>(K, row_stride, M, N, stats_out, sums);
  k_fp_finish<256><<<1, 256, 0, s>>>(sums, M, (double)M * N, stats_out, 1);
  k_fp_center<256><<<M, 256, 0, s>>>(K, row_stride, M, N, stats_out, work);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  Batch b{};
  b.shape = sh;
  b.nc = 1;
  b.cand = ident;
  b.frames = work;
  b.dtype = 0;
  b.frame_stride = (int64_t)M * N;
  b.row_stride = N;
  b.inter = inter;
  b.norm_part = reinterpret_cast<double2*>(sums);
  b.twM = twM;
  b.twN = twN;
  err = launch_warp_rowfft(b, s);
  if (err != hipSuccess) return err;
  return dispatch_cols(b, s, FK);
}

}  // namespace prnu
