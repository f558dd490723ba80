// Search kernels for gfx950: per batch of candidates, the correlation surface of
// Eq. (1) near zero shift and the PCE of Eq. (3).
//
//   k_warp_rowfft   inverse warp of the residual (Eq. 4, similarity form, bilinear,
//                   zero outside) fused with the row DFT: two warped rows form one
//                   complex row, transformed in LDS and split into the two half
//                   spectra.  Packed half-spectrum layout per row: slot 0 holds the
//                   two real bins (DC, Nyquist), slots 1..N/2-1 the complex bins.
//                   Also the FP64 sums of the warped values and of their squares
//                   (norm of Eq. 1), from bin 0 and the energy of the row transform.
//   k_col_product   column DFT of a strip of the packed half spectrum, product with
//                   the conjugated residual spectrum, FP64 Parseval energy of the
//                   product (all-shift energy of Eq. 3), inverse column DFT; only the
//                   rows |dy| <= R + 5 (peak search + exclusion reach) are stored.
//   k_band_rowifft  inverse row DFT of pairs of stored rows (Hermitian-extended);
//                   only the columns |dx| <= R + 5 are stored.
//   k_pce           signed peak over |dy|,|dx| <= R, FP64 energy of the 11x11
//                   exclusion block, PCE and NCC at the peak.
//
// Frames smaller than the fingerprint (M - ey rows, N - ex columns) are zero-padded to
// its size; the stored rows and columns then reach from -R - 5 to ey + R + 5 and
// ex + R + 5, and the peak is sought from -R to ey + R and ex + R.
//
// All transforms are unnormalised; the 1/(MN) factors are applied in FP64 in k_pce.
#include <math.h>

#include <type_traits>

#include "fft_exec.hpp"
#include "kernels.hpp"

namespace prnu {

namespace {

// Block sums through the per-wave slots red[]: a barrier first, so that an earlier sum's
// slots have been read, unless FRESH (the tile's only sum, and an earlier tile of the
// workgroup ended with a barrier).
template <int T, bool FRESH = false>
__device__ inline double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  constexpr int W = (T + 63) / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if constexpr (!FRESH) __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < W; ++i) s += red[i];
  }
  return s;  // valid in thread 0
}

// Two sums reduced together.
template <int T, bool FRESH = false>
__device__ inline double2 block_sum2(double a, double b, double2* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  constexpr int W = (T + 63) / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if constexpr (!FRESH) __syncthreads();
  if (lane == 0) red[w] = make_double2(a, b);
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < W; ++i) {
      s.x += red[i].x;
      s.y += red[i].y;
    }
  }
  return s;  // valid in thread 0
}

// Global-memory views of the device buffers: the pointers arrive inside structures, so
// without the address space the compiler emits flat accesses with 64-bit vector
// addresses.  With it, an access from a workgroup-uniform base and a 32-bit byte offset
// takes the scalar-base + vector-offset form.
typedef const __attribute__((address_space(1))) char gc_char;
typedef __attribute__((address_space(1))) char g_char;

typedef const __attribute__((address_space(1))) float gc_float;
typedef __attribute__((address_space(1))) float g_float;
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) f4v g_f4v;
// The four taps of a staged frame's entry pair: 16 bytes at 8-byte alignment (f32), or
// 8 bytes at 4-byte alignment (bf16).
typedef f4v f4v_a8 __attribute__((aligned(8)));
typedef const __attribute__((address_space(1))) f4v_a8 gc_taps32;
typedef unsigned short us4v __attribute__((ext_vector_type(4)));
typedef us4v us4v_a4 __attribute__((aligned(4)));
typedef const __attribute__((address_space(1))) us4v_a4 gc_taps16;

// Complex element at byte offset boff (8-byte aligned) from a uniform base.
template <class E>
__device__ __forceinline__ E ldo(const void* base, unsigned boff) {
  static_assert(sizeof(E) == 8, "complex elements only");
  gc_float* p = (gc_float*)((gc_char*)base + boff);
  return E{p[0], p[1]};
}
// Raw-buffer view of a workgroup-uniform block of `bytes` bytes: a load takes a 32-bit
// vector byte offset plus a scalar byte offset, so loads that differ by compile-time
// strides share one vector offset and cost no vector address arithmetic (the scalar-base
// global form only has a 13-bit immediate).  The descriptor's record count bounds the
// accesses (dword 3 is the gfx9 raw-buffer format).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_view(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ c32 ldb(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(c32, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

template <class E>
__device__ __forceinline__ void sto(void* base, unsigned boff, E v) {
  static_assert(sizeof(E) == 8, "complex elements only");
  g_float* p = (g_float*)((g_char*)base + boff);
  p[0] = v.x;
  p[1] = v.y;
}

// The four bilinear taps of the residual at B(q) = [[a, -b], [b, a]] (q - c) + c and
// the fractional offsets: one load of the staged frame's entries (x, y) and (x + 1, y),
// which hold the taps (x, y), (x, y + 1), (x + 1, y), (x + 1, y + 1).  The caller passes
// the sampling point shifted by (+1, +1): clamped to [0, N + 1] x [0, M + 1] it is
// non-negative, so truncation is the floor, and the fractions come from v_fract exactly.
// A point beyond the clamp range has all four taps outside the image; the clamped point
// then lands on border zeros with zero fractions, so the result is the same zero.  Taps
// outside the image read the zero border of the staged frame.  b0 is the frame base
// advanced to the entry of the shifted origin (pixel (-1, -1) of the image, bordered
// position (kBorder - 1, kBorder - 1)).
struct Taps {
  float w00, w01, w10, w11, fx, fy;
};

// xmax = frame width + 1, ymax = frame height + 1, RB = bytes per row of entries.
// bf16 taps are returned as stored (without the frame's scale): the scale is a power of
// two, so scaling the combined sample instead of the four taps gives the same bits.
template <int DT>
__device__ __forceinline__ Taps gather(gc_char* b0, float xmax, float ymax, unsigned RB, float xr, float yr) {
  constexpr unsigned ES = DT == 1 ? 2 : 4;
  const float xs = __builtin_amdgcn_fmed3f(xr, 0.f, xmax);
  const float ys = __builtin_amdgcn_fmed3f(yr, 0.f, ymax);
  const unsigned ix = (unsigned)xs, iy = (unsigned)ys;
  Taps t;
  t.fx = __builtin_amdgcn_fractf(xs);
  t.fy = __builtin_amdgcn_fractf(ys);
  const unsigned off = __umul24(iy, RB) + ix * (2 * ES);
  if constexpr (DT == 0) {
    const f4v q = *(gc_taps32*)(b0 + off);
    t.w00 = q.x;
    t.w10 = q.y;
    t.w01 = q.z;
    t.w11 = q.w;
  } else {
    const us4v q = *(gc_taps16*)(b0 + off);
    t.w00 = __uint_as_float((unsigned)q.x << 16);
    t.w10 = __uint_as_float((unsigned)q.y << 16);
    t.w01 = __uint_as_float((unsigned)q.z << 16);
    t.w11 = __uint_as_float((unsigned)q.w << 16);
  }
  return t;
}

// Candidates of a device-counted launch: the chunk [dyn_start, dyn_start + nc) of a list
// whose length the device wrote to *nc_dev.
__device__ __forceinline__ int dyn_count(const Batch& bt) {
  const int left = *bt.nc_dev - bt.dyn_start;
  return left < 0 ? 0 : (left < bt.nc ? left : bt.nc);
}

// A workgroup-uniform value kept in a scalar register.  The tile index of a
// grid-strided loop is uniform, but without this the compiler treats what is derived
// from it (candidate slot, frame and fingerprint pointers) as per-lane: the buffer
// descriptors built from those pointers then need a waterfall loop around every load.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform(float v) { return __int_as_float(uniform(__float_as_int(v))); }
// The same for a pointer loaded from a table (in a device-counted launch the table's
// pointer is opaque, so the compiler loads its entries per lane).
template <class P>
__device__ __forceinline__ P* uniform(P* p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v >> 32));
  return reinterpret_cast<P*>(((unsigned long long)hi << 32) | lo);
}

// The batch description for one tile of a device-counted launch.  Without it the
// compiler hoists every load that does not change from tile to tile (the twiddle
// tables' entries above all) out of the tile loop and keeps it live across the whole
// loop, which spills.  The empty asm statements make each pointer opaque, so loads
// through it stay inside the tile.
template <class P>
__device__ __forceinline__ void opaque(P*& p) {
  asm volatile("" : "+s"(p));
}
// The thread index, opaque in the same way (lane offsets and LDS addresses are
// recomputed per tile instead of held across the loop).
template <int T>
__device__ __forceinline__ int lane_id() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}
__device__ __forceinline__ Batch fresh(const Batch& bt) {
  Batch b = bt;
  opaque(b.cand);
  opaque(b.frames);
  opaque(b.fps);
  opaque(b.inter);
  opaque(b.band);
  opaque(b.win);
  opaque(b.norm_part);
  opaque(b.energy_part);
  opaque(b.rec);
  opaque(b.twM);
  opaque(b.twMi);
  opaque(b.twN);
  return b;
}

// Position of the spectrum's natural index -k (mod M) given the position x of index k.
template <class RS>
__device__ __forceinline__ int spectrum_neg(int x) {
  if constexpr (RS::pfa) {
    return RS::crt_neg(x);
  } else {
    return x == 0 ? 0 : RS::product() - x;
  }
}

// Bilinear combination; with zero fractions it returns w00 exactly.
__device__ __forceinline__ float combine(const Taps& t) {
  const float top = fmaf(t.fx, t.w01 - t.w00, t.w00);
  const float bot = fmaf(t.fx, t.w11 - t.w10, t.w10);
  return fmaf(t.fy, bot - top, top);
}

// ---------------------------------------------------------------------------

// PAD: the frames are smaller than the transform (shape.Mf() x shape.Nf()); the warp
// acts about the frame's centre and rows or columns past the frame are zero.  Without
// PAD the frame geometry is the transform's, known at compile time.
// One tile (candidate, row pair) w of nc candidates.
// DYN: called from a device-counted launch, whose table pointers are opaque (the entries
// it loads are made uniform explicitly).
template <int N, int T, int DT, bool PROJ, bool PAD, bool DYN = false>
__device__ __forceinline__ void warp_rowfft_tile(const Batch& bt, const int nc, const int tile, const int tid) {
  using RS = typename RowPlan<N>::RS;
  using P0 = Pass<RS, 0, 1, T>;
  __shared__ c32 buf[lds_size<1>(N)];
  __shared__ double2 red[(T + 63) / 64];
  const int nt = bt.shape.row_pairs();
  const int ci = bt.order ? tile / nt : tile % nc;
  const int pair = bt.order ? tile % nt : tile / nc;
  const int M = bt.shape.M;
  CandParam cp = bt.cand[ci];
  if constexpr (DYN) {
    cp.a = uniform(cp.a);
    cp.b = uniform(cp.b);
    cp.frame = uniform(cp.frame);
  }
  const int y0 = 2 * pair, y1 = y0 + 1;
  const bool has1 = y1 < M;
  // frame geometry: the transform's, or the smaller frame's
  const int Mf = PAD ? bt.shape.Mf() : M, Nf = PAD ? bt.shape.Nf() : N;
  const bool in0 = !PAD || y0 < Mf, in1 = PAD ? y1 < Mf : has1;
  const float cx = 0.5f * (float)(Nf - 1), cy = 0.5f * (float)(Mf - 1);
  FrameRef fr = bt.frames[cp.frame];
  if constexpr (DYN) fr = FrameRef{uniform(fr.data), uniform(fr.scale)};
  const float scale = (DT == 1) ? *fr.scale : 1.f;
  constexpr unsigned ES = DT == 1 ? 2 : 4;
  const unsigned NP = PAD ? (unsigned)padded_row(Nf) : (unsigned)padded_row(N);
  const unsigned RB = NP * 2 * ES;
  gc_char* b0 = (gc_char*)fr.data + (kBorder - 1) * (NP + 1) * 2 * ES;
  // Row constants of the sampling point shifted by (+1, +1).  A row outside the frame
  // (the missing second row of an odd M, or a padding row) samples far above the
  // image: clamped, it reads border zeros with zero fractions and yields exact zeros,
  // with no branch around its loads.  Padding columns do the same per sample.
  const float uy0 = (float)y0 - cy, uy1 = (float)y1 - cy;
  const float kx0 = fmaf(-cp.b, uy0, cx + 1.f), ky0 = in0 ? fmaf(cp.a, uy0, cy + 1.f) : -1e30f;
  const float kx1 = fmaf(-cp.b, uy1, cx + 1.f), ky1 = in1 ? fmaf(cp.a, uy1, cy + 1.f) : -1e30f;
  const float xmax = (float)(Nf + 1), ymax = (float)(Mf + 1);
  // General transforms: the row parts of the homogeneous coordinates.  A point whose
  // homogeneous coordinate is not positive (beyond the horizon), and a row outside the
  // frame (homogeneous coordinate -inf whatever the column), sample far above the image
  // and read zeros.
  float g00 = 0.f, g10 = 0.f, g20 = 0.f, hx0 = 0.f, hy0 = 0.f, hz0 = 0.f, hx1 = 0.f, hy1 = 0.f, hz1 = 0.f;
  if constexpr (PROJ) {
    const float* g = bt.proj + (size_t)ci * 9;
    g00 = g[0];
    g10 = g[3];
    g20 = g[6];
    hx0 = fmaf(g[1], uy0, g[2]);
    hy0 = fmaf(g[4], uy0, g[5]);
    hz0 = in0 ? fmaf(g[7], uy0, g[8]) : -INFINITY;
    hx1 = fmaf(g[1], uy1, g[2]);
    hy1 = fmaf(g[4], uy1, g[5]);
    hz1 = in1 ? fmaf(g[7], uy1, g[8]) : -INFINITY;
  }
  auto point = [&](float ux, float hx, float hy, float hz, float& xs, float& ys) {
    const float X = fmaf(g00, ux, hx), Y = fmaf(g10, ux, hy), Z = fmaf(g20, ux, hz);
    const float rz = __builtin_amdgcn_rcpf(Z);
    const bool ok = Z > 0.f;
    xs = ok ? fmaf(X, rz, cx + 1.f) : -1e30f;
    ys = ok ? fmaf(Y, rz, cy + 1.f) : -1e30f;
  };
  // The warped samples of the two rows, gathered straight into the first pass's
  // butterflies (element x = j + q NB of butterfly j), U columns at a time so that the
  // tap loads of a group are in flight together.
  // The second pass's twiddles, copied to LDS (their loads go out with the gather's;
  // the barrier after the first pass's stores makes them visible): the row kernel's
  // vector-memory pipeline then carries only the taps and the last pass's twiddles.
  using P1 = Pass<RS, 1, 1, T>;
  constexpr int TW1 = P1::NS > 1 ? P1::NS * (P1::R - 1) : 1;
  __shared__ c32 tw1[TW1];
  if constexpr (P1::NS > 1) {
    for (int i = tid; i < TW1; i += T) tw1[i] = tw_load(bt.twN, P1::TWOFF + i);
  }
  c32 v[P0::ROUNDS][P0::R];
  constexpr int U = P0::R % 6 == 0 ? 6 : (P0::R % 5 == 0 ? 5 : 4);
#pragma unroll
  for (int r = 0; r < P0::ROUNDS; ++r) {
    const int j = tid + r * T;
    const bool act = P0::full() || j < P0::TOT;
    const float uj = (float)j - cx;
#pragma unroll
    for (int q0 = 0; q0 < P0::R; q0 += U) {
      Taps t0[U], t1[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + u;
        if (q < P0::R && act) {
          const float ux = uj + (float)(q * P0::NB);
          float xa, ya, xb, yb;
          if constexpr (PROJ) {
            point(ux, hx0, hy0, hz0, xa, ya);
            point(ux, hx1, hy1, hz1, xb, yb);
          } else {
            xa = fmaf(cp.a, ux, kx0);
            ya = fmaf(cp.b, ux, ky0);
            xb = fmaf(cp.a, ux, kx1);
            yb = fmaf(cp.b, ux, ky1);
          }
          if constexpr (PAD) {
            const bool xin = j + q * P0::NB < Nf;
            ya = xin ? ya : -1e30f;
            yb = xin ? yb : -1e30f;
          }
          t0[u] = gather<DT>(b0, xmax, ymax, RB, xa, ya);
          t1[u] = gather<DT>(b0, xmax, ymax, RB, xb, yb);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + u;
        if (q < P0::R && act) {
          const float r0 = DT == 1 ? combine(t0[u]) * scale : combine(t0[u]);
          const float r1 = DT == 1 ? combine(t1[u]) * scale : combine(t1[u]);
          v[r][q] = c32{r0, r1};
          // Compiler fence holding the finished samples: this group's taps die here and
          // the next group's loads are issued after it, bounding the live registers.
          asm volatile("" ::"v"(r0), "v"(r1) : "memory");
        }
      }
    }
  }
  pass_compute<P0, 1, T, false>(v, bt.twN, tid);
  lds_store<P0, 1, T>(buf, v, tid);
  __syncthreads();
  lds_pass_own<P1, 1, T, false>(buf, tw1, tid);
  lds_passes<RS, 2, RS::count, 1, T, false>(buf, bt.twN, tid);
  // Split the transform of (row y0) + i (row y1) into the two half spectra, each stored
  // at twice its DFT: bins 1..N/2-1 as Z[k] + conj(Z[N-k]) (row y0) and
  // -i (Z[k] - conj(Z[N-k])) (row y1) without the halving, the real bins 0 and N/2
  // (packed in slot 0) doubled to match.  The factor is a power of two, so every later
  // fp32 result is exactly the unscaled one times 2 (spectra), 4 (correlation) or 16
  // (energies); the PCE kernel divides it out exactly.
  constexpr int Nh = N / 2;
  constexpr int CW = kColStrip;
  // strip-tiled: element (y0, k) at (k / CW) M CW + y0 CW + k % CW, row y1 CW further
  // The sums for the norm of Eq. (1) come from the same transform: the sum of the two
  // rows' samples is the real plus the imaginary part of bin 0, and the sum of their
  // squares is the energy of all N bins over N (Parseval); each thread sums its bins'
  // energy per iteration in fp32 and the iterations in FP64.
  // Each thread splits bins k and k + 1 (k even; they are adjacent in a strip) and
  // stores each row's pair of results as one 16-byte store.
  static_assert(Nh % 2 == 0 && CW % 2 == 0, "bin pairs stay inside a strip");
  g_char* ob = (g_char*)(bt.inter + (size_t)ci * M * tiled_cols(bt.shape) + (size_t)y0 * CW);
  const unsigned sstep = (unsigned)M * CW;
  double s1 = 0.0, s2 = 0.0;
  for (int kp = tid; kp < Nh / 2; kp += T) {
    const int k = 2 * kp;
    const c32 z0 = buf[lds_slot<1>(k)], z1 = buf[lds_slot<1>(k + 1)];
    const c32 m1 = buf[lds_slot<1>(N - k - 1)];  // the partner of bin k + 1
    c32 a0, b0;                                  // bin k of rows y0 and y1
    float e;
    if (k == 0) {
      const c32 zh = buf[lds_slot<1>(Nh)];
      a0 = c32{z0.x + z0.x, zh.x + zh.x};
      b0 = c32{z0.y + z0.y, zh.y + zh.y};
      e = fmaf(z0.x, z0.x, fmaf(z0.y, z0.y, fmaf(zh.x, zh.x, zh.y * zh.y)));
      s1 = (double)z0.x + (double)z0.y;
    } else {
      const c32 m0 = buf[lds_slot<1>(N - k)];
      a0 = c32{z0.x + m0.x, z0.y - m0.y};
      b0 = c32{z0.y + m0.y, m0.x - z0.x};
      e = fmaf(z0.x, z0.x, fmaf(z0.y, z0.y, fmaf(m0.x, m0.x, m0.y * m0.y)));
    }
    const c32 a1 = {z1.x + m1.x, z1.y - m1.y}, b1 = {z1.y + m1.y, m1.x - z1.x};
    e = fmaf(z1.x, z1.x, fmaf(z1.y, z1.y, fmaf(m1.x, m1.x, fmaf(m1.y, m1.y, e))));
    s2 += (double)e;
    const unsigned o = (__umul24((unsigned)k / CW, sstep) + (unsigned)k % CW) * 8u;
    *(g_f4v*)(ob + o) = f4v{a0.x, a0.y, a1.x, a1.y};
    if (has1) *(g_f4v*)(ob + o + CW * 8u) = f4v{b0.x, b0.y, b1.x, b1.y};
  }
  const double2 s12 = block_sum2<T, true>(s1, s2 * (1.0 / (double)N), red);
  if (tid == 0) bt.norm_part[(size_t)ci * bt.shape.row_pairs() + pair] = s12;
}

template <int N, int T, int DT, bool PROJ, bool PAD>
__global__ __launch_bounds__(T, 4) void k_warp_rowfft(Batch bt) {
  warp_rowfft_tile<N, T, DT, PROJ, PAD>(bt, bt.nc, (int)blockIdx.x, (int)threadIdx.x);
}

// Device-counted form: the candidate count is read from device memory and a fixed grid
// strides over the tiles (an empty count costs one pass of the grid's workgroups).
template <int N, int T, int DT, bool PROJ, bool PAD>
__global__ __launch_bounds__(T, 4) void k_warp_rowfft_dyn(Batch bt) {
  const int nc = dyn_count(bt), total = nc * bt.shape.row_pairs();
  for (int w = (int)blockIdx.x; w < total; w += (int)gridDim.x) {
    warp_rowfft_tile<N, T, DT, PROJ, PAD, true>(fresh(bt), uniform(nc), uniform(w), lane_id<T>());
    __syncthreads();  // LDS is reused by the next tile
  }
}

// ---------------------------------------------------------------------------

// One tile (candidate, column strip or half strip) w of nc candidates.
template <int M, int T, bool PRODUCT, bool DYN = false>
__device__ __forceinline__ void col_tile(const Batch& bt, c32* fk_out, const int nc, const int tile, const int tid) {
  // SW columns per strip in memory; a workgroup transforms CW of them (all, or one half
  // of the strip when col_split(M) is 2), interleaved CW-wide in LDS
  constexpr int SW = kColStrip, HS = col_split(M), CW = SW / HS;
  using RS = typename ColPlan<M>::RS;
  using RI = Reverse<RS>;
  constexpr int NP = RS::count;
  using F0 = Pass<RS, 0, CW, T>;
  using FL = Pass<RS, NP - 1, CW, T>;
  using I0 = Pass<RI, 0, CW, T>;
  using IL = Pass<RI, NP - 1, CW, T>;
  // the inverse's first pass takes the forward last pass's butterflies as they are (a
  // reversed Stockham plan reads j + q NB where the forward wrote j + q Ns; a
  // prime-factor plan transforms the same dimension in place)
  static_assert(I0::R == FL::R && I0::TOT == FL::TOT && (RS::pfa || I0::NB == FL::NS),
                "inverse starts on the forward outputs");
  __shared__ c32 buf[lds_size<CW>(M * CW)];
  // column-0 exchange: its own array, or (half strips, whose LDS must stay under half a
  // CU's) the start of buf once the forward data has been read
  __shared__ c32 col0_own[PRODUCT && HS == 1 ? M : 1];
  __shared__ double red[(T + 63) / 64];
  const int nt = col_strips(bt.shape) * HS;  // col_blocks, with M known here
  const int ci = bt.order ? tile / nt : tile % nc;
  const int sb = bt.order ? tile % nt : tile / nc;
  const int strip = sb / HS, half = sb % HS;
  const int Nh = bt.shape.N / 2;
  const int c0 = strip * SW + half * CW;
  // this candidate's strip of the strip-tiled intermediate and fingerprint spectrum:
  // element (row y, column strip SW + b) at y SW + b from the strip's base; this
  // workgroup's columns start hb bytes into each row
  const size_t sbase = (size_t)strip * M * SW;
  const unsigned hb = (unsigned)(half * CW) * 8u;
  const c32* src = bt.inter + (size_t)ci * M * tiled_cols(bt.shape) + sbase;
  const c32* FK = nullptr;
  if constexpr (PRODUCT) {
    if constexpr (DYN)
      FK = uniform(bt.fps[uniform(bt.cand[ci].fp)].FK) + sbase;
    else
      FK = bt.fps[bt.cand[ci].fp].FK + sbase;
  }
  // Forward pass 0 straight from the strip in global memory (all loads issued first).
  const __amdgpu_buffer_rsrc_t srcv = buffer_view(src, (unsigned)(M * SW * 8));
  {
    c32 v[F0::ROUNDS][F0::R];
#pragma unroll
    for (int r = 0; r < F0::ROUNDS; ++r) {
      const int g = tid + r * T;
      // element (row g / CW + q NB, column c0 + g % CW) at (g / CW + q NB) SW + g % CW of
      // the strip plus the half's offset: the wave reads contiguous memory (whole rows of
      // the strip, or their halves), the per-q step is a constant.  A lane past the last
      // butterfly reads from element 0 instead, and a lane past the half spectrum reads
      // the strip's padding: their values are never stored, and no zero fill is spent
      // on them.
      unsigned o = 0u;
      if (F0::full() || g < F0::TOT) {
        if constexpr (RS::pfa) {
          // prime-factor plan: position j + q NB holds row (row of j) + q NB mod M
          o = (unsigned)(RS::in_index(g / CW) * SW + g % CW) * 8u + hb;
        } else if constexpr (HS == 1) {
          o = (unsigned)g * 8u;
        } else {
          o = (unsigned)((g / CW) * SW + g % CW) * 8u + hb;
        }
      }
      constexpr unsigned qs = (unsigned)F0::NB * SW * 8u;
#pragma unroll
      for (int q = 0; q < F0::R; ++q) {
        if constexpr (RS::pfa) {
          // the offset wrapped to the strip (min picks the unwrapped one while the
          // subtraction would go below zero); the whole offset goes in the vector
          // operand, which is what the descriptor's range check sees
          const unsigned oq = o + (unsigned)q * qs;
          v[r][q] = ldb(srcv, min(oq, oq - (unsigned)(M * SW * 8)), 0u);
        } else {
          v[r][q] = ldb(srcv, o, (unsigned)q * qs);
        }
      }
    }
    pass_compute<F0, CW, T, false>(v, bt.twM, tid);
    lds_store<F0, CW, T>(buf, v, tid);
  }
  __syncthreads();
  lds_passes<RS, 1, NP - 1, CW, T, false>(buf, bt.twM, tid);
  // Forward last pass: its outputs (row j + q Ns of column c0 + b) stay in registers.
  c32 v[FL::ROUNDS][FL::R];
  if constexpr (!PRODUCT) {
    lds_load<FL, CW, T>(buf, v, tid);
    pass_compute<FL, CW, T, false>(v, bt.twM, tid);
#pragma unroll
    for (int r = 0; r < FL::ROUNDS; ++r) {
      const int g = tid + r * T;
      const int col = c0 + g % CW, j = g / CW;
      if ((FL::full() || g < FL::TOT) && col < Nh) {
#pragma unroll
        for (int q = 0; q < FL::R; ++q) {
          const int row = FL::out_el(j, q);
          c32 x = v[r][q];
          if (row == 0 && col == 0) x.x = 0.f;  // DC of the mean-free fingerprint is exactly zero
          fk_out[sbase + (size_t)row * SW + half * CW + g % CW] = x;  // strip-tiled, like the intermediate
        }
      }
    }
  } else {
    // Fingerprint spectrum for the same elements, requested before the last pass.
    const __amdgpu_buffer_rsrc_t fkv = buffer_view(FK, (unsigned)(M * SW * 8));
    c32 fk[FL::ROUNDS][FL::R];
#pragma unroll
    for (int r = 0; r < FL::ROUNDS; ++r) {
      const int g = tid + r * T;
      // a lane past the last butterfly reads from element 0 (values never used)
      unsigned o = 0u;
      if (FL::full() || g < FL::TOT) {
        if constexpr (HS == 1)
          o = (unsigned)(FL::out_el(g / CW, 0) * CW + g % CW) * 8u;
        else
          o = (unsigned)(FL::out_el(g / CW, 0) * SW + g % CW) * 8u + hb;
      }
      constexpr unsigned qs = (unsigned)FL::NS * SW * 8u;
#pragma unroll
      for (int q = 0; q < FL::R; ++q) fk[r][q] = ldb(fkv, o, (unsigned)q * qs);
    }
    lds_load<FL, CW, T>(buf, v, tid);
    pass_compute<FL, CW, T, false>(v, bt.twM, tid);
    // Parseval energy of the product: each |G|^2 (an fp32 product of fp32 data) is
    // accumulated in FP64; bins of columns 1..N/2-1 stand for two bins of the full
    // spectrum (weight 2, applied to the sum), the two real columns packed in column 0
    // have weight 1.
    // A butterfly's R products are summed in fp32, the butterflies in FP64.
    double e = 0.0, e0 = 0.0;
#pragma unroll
    for (int r = 0; r < FL::ROUNDS; ++r) {
      const int g = tid + r * T;
      const int col = c0 + g % CW;
      if ((FL::full() || g < FL::TOT) && col < Nh && col != 0) {
        float eb = 0.f;
#pragma unroll
        for (int q = 0; q < FL::R; ++q) {
          const c32 gq = cmulc(fk[r][q], v[r][q]);
          eb = fmaf(gq.x, gq.x, fmaf(gq.y, gq.y, eb));
          v[r][q] = gq;
        }
        e += (double)eb;
      }
    }
    if (c0 == 0) {
      // Column 0 packs two real columns (x-bins 0 and N/2): split each spectrum by
      // Hermitian symmetry in ky (partner rows live in other threads: exchange through
      // LDS), multiply, and pack the two products again.
      if constexpr (HS > 1) __syncthreads();  // every thread has read its forward data from buf
      c32* col0 = static_cast<c32*>(__builtin_assume_aligned(HS > 1 ? buf : col0_own, 8));
#pragma unroll
      for (int r = 0; r < FL::ROUNDS; ++r) {
        const int g = tid + r * T;
        if ((FL::full() || g < FL::TOT) && g % CW == 0) {
#pragma unroll
          for (int q = 0; q < FL::R; ++q) col0[FL::out_el(g / CW, q)] = v[r][q];
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < FL::ROUNDS; ++r) {
        const int g = tid + r * T;
        if ((FL::full() || g < FL::TOT) && g % CW == 0) {
#pragma unroll
          for (int q = 0; q < FL::R; ++q) {
            const int ky = FL::out_el(g / CW, q);  // position of the bin
            const int kn = spectrum_neg<RS>(ky);     // position of its mirror bin
            const c32 z = v[r][q], zn = col0[kn];
            const c32 zk = fk[r][q], zkn = ldo<c32>(FK, (unsigned)kn * SW * 8u);
            const c32 A = {0.5f * (z.x + zn.x), 0.5f * (z.y - zn.y)};
            const c32 B = {0.5f * (z.y + zn.y), -0.5f * (z.x - zn.x)};
            const c32 FA = {0.5f * (zk.x + zkn.x), 0.5f * (zk.y - zkn.y)};
            const c32 FB = {0.5f * (zk.y + zkn.y), -0.5f * (zk.x - zkn.x)};
            const c32 GA = cmulc(FA, A), GB = cmulc(FB, B);
            e0 += (double)fmaf(GA.x, GA.x, GA.y * GA.y) + (double)fmaf(GB.x, GB.x, GB.y * GB.y);
            v[r][q] = c32{GA.x - GB.y, GA.y + GB.x};  // GA + i GB
          }
        }
      }
    }
    // Every thread must be done reading the forward data in LDS before the inverse's
    // first stores, unless that pass writes exactly the elements the forward last pass
    // read, butterfly by butterfly (a prime-factor plan's last dimension, transformed
    // in place, with the column-0 exchange in an array of its own).
    static_assert(!RS::pfa || (std::is_base_of<FL, I0>::value && I0::in_place), "same butterflies");
    if constexpr (!(RS::pfa && HS == 1)) __syncthreads();
    // Inverse pass 0 works on the same butterflies the forward last pass produced.
    pass_compute<I0, CW, T, true>(v, bt.twMi, tid);
    lds_store<I0, CW, T>(buf, v, tid);
    __syncthreads();
    lds_passes<RI, 1, NP - 1, CW, T, true>(buf, bt.twMi, tid);
    // Inverse last pass: keep only the rows -R-5 <= dy <= ey + R + 5 and store them to
    // the band (band row dy + R + 5).
    {
      c32 w[IL::ROUNDS][IL::R];
      lds_load<IL, CW, T>(buf, w, tid);
      pass_compute<IL, CW, T, true>(w, bt.twMi, tid);
      const int H = bt.shape.radius + 5, TOP = bt.shape.ey + H, BR = bt.shape.band_rows();
      c32* dst = bt.band + (size_t)ci * BR * Nh;
      // Output q of butterfly j is position j + q Ns (Ns = M / R).  A Stockham plan's
      // positions are rows; when the band reaches less than 2 Ns from row 0 on either
      // side, only q in {0, 1, R-2, R-1} can fall in it, and the other outputs are not
      // even tested.  In a prime-factor plan the last pass transforms dimension 0
      // (q is the coordinate n_0), so output q is row (row of j) + q M / R mod M.
      static_assert(IL::NB == IL::NS, "last pass: butterfly j writes positions j + q Ns");
      const bool narrow = !RI::pfa && IL::R >= 4 && TOP < 2 * IL::NS;
      constexpr int STEP = RI::pfa ? M / IL::R : IL::NS;
#pragma unroll
      for (int r = 0; r < IL::ROUNDS; ++r) {
        const int g = tid + r * T;
        const int col = c0 + g % CW, j = g / CW;
        if ((IL::full() || g < IL::TOT) && col < Nh) {
          const int row0 = RI::out_index(IL::out_el(j, 0));
          // prime-factor plans: the band is the cyclic interval of rows from M - H to TOP,
          // so with t0 = (row0 + H) mod M output q lands on band row (t0 + q STEP) mod M
          // when that is below BR (one wrap at most: t0 < M, q STEP < M)
          int t0 = row0 + H;
          if constexpr (RI::pfa) t0 = t0 >= M ? t0 - M : t0;
          auto put = [&](int q) {
            if constexpr (RI::pfa) {
              int br = t0 + q * STEP;
              br = br >= M ? br - M : br;
              if (br < BR) sto<c32>(dst, (__umul24((unsigned)br, (unsigned)Nh) + (unsigned)col) * 8u, w[r][q]);
            } else {
              const int row = row0 + q * STEP;
              const int br = row <= TOP ? row + H : row - (M - H);
              if (row <= TOP || row >= M - H) sto<c32>(dst, (__umul24((unsigned)br, (unsigned)Nh) + (unsigned)col) * 8u, w[r][q]);
            }
          };
          if (narrow) {
            put(0);
            put(1);
            put(IL::R - 2);
            put(IL::R - 1);
          } else {
#pragma unroll
            for (int q = 0; q < IL::R; ++q) put(q);
          }
        }
      }
    }
    e = block_sum<T, true>(fma(2.0, e, e0), red);
    if (tid == 0) bt.energy_part[(size_t)ci * nt + sb] = e;
  }
}

template <int M, int T, bool PRODUCT>
__global__ __launch_bounds__(T, 4) void k_col(Batch bt, c32* fk_out) {
  col_tile<M, T, PRODUCT>(bt, fk_out, bt.nc, (int)blockIdx.x, (int)threadIdx.x);
}

template <int M, int T>
__global__ __launch_bounds__(T, 4) void k_col_dyn(Batch bt) {
  const int nc = dyn_count(bt), total = nc * col_blocks(bt.shape);
  for (int w = (int)blockIdx.x; w < total; w += (int)gridDim.x) {
    col_tile<M, T, true, true>(fresh(bt), nullptr, uniform(nc), uniform(w), lane_id<T>());
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------

// One tile (candidate, pair of band rows) w of nc candidates.
template <int N, int T>
__device__ __forceinline__ void band_rowifft_tile(const Batch& bt, const int nc, const int tile, const int tid) {
  using RS = typename RowPlan<N>::RS;
  constexpr int NP = RS::count;
  using P0 = Pass<RS, 0, 1, T>;
  using PL = Pass<RS, NP - 1, 1, T>;
  __shared__ c32 buf[lds_size<1>(N)];
  constexpr int Nh = N / 2;
  const int ci = tile % nc;
  const int p = tile / nc;
  const int H = bt.shape.radius + 5, BR = bt.shape.band_rows(), BX = bt.shape.win_cols(), RGT = bt.shape.ex + H;
  const int ra = 2 * p, rb = ra + 1;
  const bool hasb = rb < BR;
  const c32* ba = bt.band + ((size_t)ci * BR + ra) * Nh;
  // The two band rows staged in LDS (rows a and b side by side, 16-byte loads; the
  // Hermitian extension below reads every element twice, from LDS).  Nh is even and
  // each band row starts 16-byte aligned.
  static_assert(N % 4 == 0, "band rows in 16-byte pairs");
  {
    const __attribute__((address_space(1))) f4v* ga = (const __attribute__((address_space(1))) f4v*)ba;
    for (int i = tid; i < Nh; i += T) {
      const f4v x = (i < Nh / 2 || hasb) ? ga[i] : f4v{0.f, 0.f, 0.f, 0.f};
      buf[2 * i] = c32{x.x, x.y};
      buf[2 * i + 1] = c32{x.z, x.w};
    }
  }
  __syncthreads();
  const c32* sa = buf;
  const c32* sb = buf + Nh;
  // Pass 0 inputs from the staged band rows, Hermitian-extended: element kx of
  // (row a) + i (row b), where bin k > N/2 is the conjugate of bin N - k and bins 0 and
  // N/2 (both real) are packed in slot 0.  For each unrolled (round, q) the span of kx
  // over the round's butterflies is a compile-time range: wholly below N/2 (direct
  // reads), wholly above (mirrored reads, conjugated), or straddling it (per-lane
  // selection); the packed bins need a per-lane test only where they fall in the span.
  {
    c32 la[P0::ROUNDS][P0::R], lb[P0::ROUNDS][P0::R];
#pragma unroll
    for (int r = 0; r < P0::ROUNDS; ++r) {
      const int j = tid + r * T;
      const bool act = P0::full() || j < P0::TOT;
#pragma unroll
      for (int q = 0; q < P0::R; ++q) {
        const int lo = r * T + q * P0::NB;
        const int hi = (P0::TOT < r * T + T ? P0::TOT : r * T + T) - 1 + q * P0::NB;
        const int kx = P0::in_el(j, q);
        int sx;
        if (hi < Nh)
          sx = kx;
        else if (lo > Nh)
          sx = N - kx;
        else
          sx = kx <= Nh ? (kx == Nh ? 0 : kx) : N - kx;
        const int x = act ? sx : 0;
        la[r][q] = sa[x];
        lb[r][q] = sb[x];
      }
    }
    __syncthreads();  // every staged element read before pass 0 stores over them
    c32 v[P0::ROUNDS][P0::R];
#pragma unroll
    for (int r = 0; r < P0::ROUNDS; ++r) {
      const int j = tid + r * T;
#pragma unroll
      for (int q = 0; q < P0::R; ++q) {
        const int lo = r * T + q * P0::NB;
        const int hi = (P0::TOT < r * T + T ? P0::TOT : r * T + T) - 1 + q * P0::NB;
        const int kx = P0::in_el(j, q);
        c32 ca = la[r][q], cb = lb[r][q];
        if (lo > Nh) {
          ca = cconj(ca);
          cb = cconj(cb);
        } else if (hi >= Nh || lo == 0) {
          if (kx == 0) {
            ca = c32{ca.x, 0.f};
            cb = c32{cb.x, 0.f};
          } else if (kx == Nh) {
            ca = c32{ca.y, 0.f};
            cb = c32{cb.y, 0.f};
          } else if (kx > Nh) {
            ca = cconj(ca);
            cb = cconj(cb);
          }
        }
        v[r][q] = c32{ca.x - cb.y, ca.y + cb.x};  // ca + i cb
      }
    }
    pass_compute<P0, 1, T, true>(v, bt.twN, tid);
    lds_store<P0, 1, T>(buf, v, tid);
  }
  __syncthreads();
  lds_passes<RS, 1, NP - 1, 1, T, true>(buf, bt.twN, tid);
  // Last pass in registers; keep the columns -R-5 <= dx <= ex + R + 5 (window column
  // dx + R + 5).
  c32 w[PL::ROUNDS][PL::R];
  lds_load<PL, 1, T>(buf, w, tid);
  pass_compute<PL, 1, T, true>(w, bt.twN, tid);
  float* wa = bt.win + ((size_t)ci * BR + ra) * BX;
  float* wb = wa + BX;
  // Output q of butterfly j is column j + q Ns (Ns = N / R): as for the band rows, a
  // window narrower than 2 Ns on either side can only hold q in {0, 1, R-2, R-1}.
  static_assert(PL::NB == PL::NS, "last pass: butterfly j writes columns j + q Ns");
  const bool narrow = PL::R >= 4 && RGT < 2 * PL::NS;
#pragma unroll
  for (int r = 0; r < PL::ROUNDS; ++r) {
    const int j = tid + r * T;
    if (PL::full() || j < PL::TOT) {
      auto put = [&](int q) {
        const int x = PL::out_el(j, q);
        const int wi = x <= RGT ? x + H : x - (N - H);
        if (x <= RGT || x >= N - H) {
          wa[wi] = w[r][q].x;
          if (hasb) wb[wi] = w[r][q].y;
        }
      };
      if (narrow) {
        put(0);
        put(1);
        put(PL::R - 2);
        put(PL::R - 1);
      } else {
#pragma unroll
        for (int q = 0; q < PL::R; ++q) put(q);
      }
    }
  }
}

template <int N, int T>
__global__ __launch_bounds__(T) void k_band_rowifft(Batch bt) {
  band_rowifft_tile<N, T>(bt, bt.nc, (int)blockIdx.x, (int)threadIdx.x);
}

template <int N, int T>
__global__ __launch_bounds__(T) void k_band_rowifft_dyn(Batch bt) {
  const int nc = dyn_count(bt), total = nc * bt.shape.band_pairs();
  for (int w = (int)blockIdx.x; w < total; w += (int)gridDim.x) {
    band_rowifft_tile<N, T>(fresh(bt), uniform(nc), uniform(w), lane_id<T>());
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------

// PCE of candidate ci.
template <int T>
__device__ __forceinline__ void pce_tile(const Batch& bt, const int ci) {
  __shared__ double red[(T + 63) / 64];
  __shared__ float sbest[(T + 63) / 64];
  __shared__ int sidx[(T + 63) / 64];
  __shared__ int peak_idx;
  // peak search over SY x SX shifts (-R..ey+R by -R..ex+R), in a window of BR x BX
  const int R = bt.shape.radius, BR = bt.shape.band_rows(), BX = bt.shape.win_cols();
  const int SY = bt.shape.ey + 2 * R + 1, SX = bt.shape.ex + 2 * R + 1, SS = SY * SX;
  const float* w = bt.win + (size_t)ci * BR * BX;
  float best = -INFINITY;
  int bidx = 0x7fffffff;
  constexpr int G = 16;  // window values loaded per thread before they are compared
  for (int base = 0; base < SS; base += G * T) {
    float v[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int idx = base + threadIdx.x + g * T;
      const int r = idx / SX, c = idx % SX;
      v[g] = idx < SS ? w[(r + 5) * BX + (c + 5)] : -INFINITY;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int idx = base + threadIdx.x + g * T;
      if (idx < SS && v[g] > best) {  // indices increase per thread: the first maximum is kept
        best = v[g];
        bidx = idx;
      }
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
  const int pr = found ? pidx / SX : R, pc = found ? pidx % SX : R;
  // energy of the exclusion block (its centre is at window (pr + 5, pc + 5))
  double sd = 0.0;
  if (threadIdx.x < 121) {
    const int a = threadIdx.x / 11 - 5, b = threadIdx.x % 11 - 5;
    const double v = (double)w[(pr + 5 + a) * BX + (pc + 5 + b)];
    sd = v * v;
  }
  sd = block_sum<T>(sd, red);
  const int nstrips = col_blocks(bt.shape);
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
    // Both spectra are stored at twice the DFT (row kernel): the window holds 4 MN C and
    // the energies 16 (MN)^2 C^2 (Parseval: 16 MN sum C^2); the divisions are exact.
    const double MN = (double)bt.shape.M * (double)bt.shape.N;
    const double cpk = (double)sbest[0] / (4.0 * MN);      // C at the peak
    const double all = e / (16.0 * MN);                    // sum over all shifts of C^2 (Parseval)
    const double excl = sd / (16.0 * MN * MN);             // sum over the exclusion block
    const double off = all - excl;
    CandRecord r;
    r.pce = (found && off > 0.0) ? copysign(cpk * cpk, cpk) * (MN - 121.0) / off : (found ? 0.0 : NAN);
    const double rn2 = s2 - s1 * s1 / MN;
    const double fpn = bt.fps[bt.cand[ci].fp].norm;
    r.rho = (rn2 > 0.0 && fpn > 0.0) ? cpk / (fpn * sqrt(rn2)) : 0.0;
    r.peak = cpk;
    r.dx = pc - R;
    r.dy = pr - R;
    bt.rec[ci] = r;
  }
}

template <int T>
__global__ __launch_bounds__(T) void k_pce(Batch bt) {
  pce_tile<T>(bt, (int)blockIdx.x);
}

template <int T>
__global__ __launch_bounds__(T) void k_pce_dyn(Batch bt) {
  const int nc = dyn_count(bt);
  for (int ci = (int)blockIdx.x; ci < nc; ci += (int)gridDim.x) {
    pce_tile<T>(fresh(bt), uniform(ci));
    __syncthreads();
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

// K - mean into the staged layout (one block per row of entries).
template <int T>
__global__ __launch_bounds__(T) void k_fp_center(const float* K, int64_t rs, int M, int N, const double* mean,
                                                 float* out) {
  const int y0 = (int)blockIdx.x - kBorder, y1 = y0 + 1;
  const double mu = *mean;
  const int64_t np = padded_row(N);
  float* row = out + (int64_t)blockIdx.x * np * 2;
  for (int x = (int)threadIdx.x - kBorder; x < N + kBorder; x += T) {
    const bool xin = x >= 0 && x < N;
    const bool in0 = xin && y0 >= 0 && y0 < M, in1 = xin && y1 >= 0 && y1 < M;
    row[2 * (x + kBorder)] = in0 ? (float)((double)K[(int64_t)y0 * rs + x] - mu) : 0.f;
    row[2 * (x + kBorder) + 1] = in1 ? (float)((double)K[(int64_t)y1 * rs + x] - mu) : 0.f;
  }
}

// Frames into the staged layout (one block per row of entries of one frame).
template <int T, typename E>
__global__ __launch_bounds__(T) void k_pad_frames(const E* src, int64_t sfs, int64_t srs, int M, int N, E* dst) {
  const int f = blockIdx.y;
  const int y0 = (int)blockIdx.x - kBorder, y1 = y0 + 1;
  const int64_t np = padded_row(N);
  E* row = dst + (int64_t)f * padded_frame(M, N) + (int64_t)blockIdx.x * np * 2;
  auto clampy = [&](int y) { return (int64_t)(y < 0 ? 0 : (y < M ? y : M - 1)); };
  const E* s0 = src + (int64_t)f * sfs + clampy(y0) * srs;
  const E* s1 = src + (int64_t)f * sfs + clampy(y1) * srs;
  const bool r0 = y0 >= 0 && y0 < M, r1 = y1 >= 0 && y1 < M;
  for (int x = (int)threadIdx.x - kBorder; x < N + kBorder; x += T) {
    const bool xin = x >= 0 && x < N;
    row[2 * (x + kBorder)] = (xin && r0) ? s0[x] : E(0);
    row[2 * (x + kBorder) + 1] = (xin && r1) ? s1[x] : E(0);
  }
}

// ---------------------------------------------------------------------------
// Dispatch.

template <int N>
constexpr int row_threads() {
  return N >= 3840 ? 256 : (N >= 1280 ? 128 : 64);
}
template <int M>
constexpr int col_threads() {
  return M >= 1920 || M == 1080 || M == 720 ? 512 : 256;
}

// Workgroups of a device-counted launch of a chunk of `tiles` tiles: one per tile
// (full), or per_cu per CU striding over them, capped by the tiles.  Striding
// workgroups stay resident for several tiles, whose barriers then hold the CU's other
// waves; with 128 row or band workgroups (16 column workgroups of 512 threads) per CU a
// tile costs 7% (row kernel) to 20% (column kernel) more than in a one-tile workgroup,
// against 30% and more with one or two residencies per CU.
inline unsigned dyn_grid(const Batch& b, int64_t tiles, int per_cu) {
  const int64_t g = b.dyn_full ? tiles : (int64_t)256 * per_cu;
  return (unsigned)(tiles < g ? (tiles > 0 ? tiles : 1) : g);
}

template <int N, int T, int DT>
void launch_rows_dt(const Batch& b, dim3 grid, hipStream_t s) {
  if (b.nc_dev) {
    // device-counted launches carry similarity candidates only
    const dim3 g(dyn_grid(b, (int64_t)b.nc * b.shape.row_pairs(), 128));
    if (b.shape.padded())
      k_warp_rowfft_dyn<N, T, DT, false, true><<<g, T, 0, s>>>(b);
    else
      k_warp_rowfft_dyn<N, T, DT, false, false><<<g, T, 0, s>>>(b);
  } else if (b.proj) {
    if (b.shape.padded())
      k_warp_rowfft<N, T, DT, true, true><<<grid, T, 0, s>>>(b);
    else
      k_warp_rowfft<N, T, DT, true, false><<<grid, T, 0, s>>>(b);
  } else if (b.shape.padded()) {
    k_warp_rowfft<N, T, DT, false, true><<<grid, T, 0, s>>>(b);
  } else {
    k_warp_rowfft<N, T, DT, false, false><<<grid, T, 0, s>>>(b);
  }
}

template <int N>
hipError_t launch_rows(const Batch& b, hipStream_t s) {
  constexpr int T = row_threads<N>();
  dim3 grid((unsigned)(b.nc * b.shape.row_pairs()));
  if (b.dtype == 1)
    launch_rows_dt<N, T, 1>(b, grid, s);
  else
    launch_rows_dt<N, T, 0>(b, grid, s);
  return hipGetLastError();
}

template <int M>
hipError_t launch_cols(const Batch& b, hipStream_t s, c32* fk_out) {
  constexpr int T = col_threads<M>();
  dim3 grid((unsigned)(b.nc * col_blocks(b.shape)));
  if (b.nc_dev)
    k_col_dyn<M, T><<<dim3(dyn_grid(b, (int64_t)b.nc * col_blocks(b.shape), 1024 / T * 16)), T, 0, s>>>(b);
  else if (fk_out)
    k_col<M, T, false><<<grid, T, 0, s>>>(b, fk_out);
  else
    k_col<M, T, true><<<grid, T, 0, s>>>(b, nullptr);
  return hipGetLastError();
}

template <int N>
hipError_t launch_band(const Batch& b, hipStream_t s) {
  constexpr int T = row_threads<N>();
  dim3 grid((unsigned)(b.nc * b.shape.band_pairs()));
  if (b.nc_dev)
    k_band_rowifft_dyn<N, T><<<dim3(dyn_grid(b, (int64_t)b.nc * b.shape.band_pairs(), 128)), T, 0, s>>>(b);
  else
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
  if (b.nc_dev)
    k_pce_dyn<256><<<dim3(dyn_grid(b, b.nc, 4)), 256, 0, s>>>(b);
  else
    k_pce<256><<<dim3((unsigned)b.nc), 256, 0, s>>>(b);
  return hipGetLastError();
}

hipError_t launch_pad_frames(const void* src, int elem_bytes, int64_t src_frame_stride, int64_t src_row_stride,
                             int n_frames, int M, int N, void* dst, hipStream_t s) {
  if (n_frames <= 0) return hipSuccess;
  dim3 grid((unsigned)pair_rows(M), (unsigned)n_frames);
  if (elem_bytes == 4)
    k_pad_frames<256, float><<<grid, 256, 0, s>>>(reinterpret_cast<const float*>(src), src_frame_stride,
                                                   src_row_stride, M, N, reinterpret_cast<float*>(dst));
  else
    k_pad_frames<256, unsigned short><<<grid, 256, 0, s>>>(reinterpret_cast<const unsigned short*>(src),
                                                            src_frame_stride, src_row_stride, M, N,
                                                            reinterpret_cast<unsigned short*>(dst));
  return hipGetLastError();
}

hipError_t launch_fp_prepare(const float* K, int64_t row_stride, const Shape& sh, float* work, c32* inter,
                             double* sums, double* stats_out, c32* FK, const c32* twM, const c32* twMi, const c32* twN,
                             const CandParam* ident, const FrameRef* wref, hipStream_t s) {
  const int M = sh.M, N = sh.N;
  k_fp_rowsums<256><<<M, 256, 0, s>>>(K, row_stride, M, N, nullptr, sums);
  k_fp_finish<256><<<1, 256, 0, s>>>(sums, M, (double)M * N, stats_out, 0);
  k_fp_rowsums<256><<<M, 256, 0, s>>>(K, row_stride, M, N, stats_out, sums);
  k_fp_finish<256><<<1, 256, 0, s>>>(sums, M, (double)M * N, stats_out, 1);
  k_fp_center<256><<<(unsigned)pair_rows(M), 256, 0, s>>>(K, row_stride, M, N, stats_out, work);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  Batch b{};
  b.shape = sh;
  b.nc = 1;
  b.cand = ident;
  b.frames = wref;
  b.dtype = 0;
  b.inter = inter;
  b.norm_part = reinterpret_cast<double2*>(sums);
  b.twM = twM;
  b.twMi = twMi;
  b.twN = twN;
  err = launch_warp_rowfft(b, s);
  if (err != hipSuccess) return err;
  return dispatch_cols(b, s, FK);
}

}  // namespace prnu
