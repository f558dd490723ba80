// Mixed-radix Stockham FFT building blocks for gfx950.
//
// The correlation of Eq. (1) is evaluated at every circular shift as a product of
// 2-D DFTs (row pass + column pass).  Every transform length used by the search is
// 2,3,5-smooth; a length L is factorised into radices r_0 r_1 ... (each 2..16) and
// computed by autosorting Stockham passes: pass p reads r_p elements spaced L/r_p
// apart, multiplies by the twiddles W_{Ns r}^{k q} (Ns = r_0 ... r_{p-1},
// k = j mod Ns), applies a radix-r DFT in registers and writes the results Ns apart
// starting at (j - k) r + k.  The output is in natural order after the last pass.
//
// Small DFTs are built at compile time: radix 2, 3, 4, 5 by hand; composite radices
// with coprime factors (6, 10, 12, 15, 18, 20, 30) by a prime-factor split, the others
// (8, 9, 16) by one Cooley-Tukey split with constant twiddles.
// Everything here is __host__ __device__ so that the same index and butterfly code can
// be exercised by a host emulator.
#pragma once

#include <hip/hip_runtime.h>

namespace prnu {

struct c32 {
  float x, y;
};

__host__ __device__ __forceinline__ c32 cadd(c32 a, c32 b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ __forceinline__ c32 csub(c32 a, c32 b) { return {a.x - b.x, a.y - b.y}; }
__host__ __device__ __forceinline__ c32 cscale(c32 a, float s) { return {a.x * s, a.y * s}; }
__host__ __device__ __forceinline__ c32 cconj(c32 a) { return {a.x, -a.y}; }
// a * b
__host__ __device__ __forceinline__ c32 cmul(c32 a, c32 b) {
  return {fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x)};
}
// a * conj(b)
__host__ __device__ __forceinline__ c32 cmulc(c32 a, c32 b) {
  return {fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y)};
}
// -i * a
__host__ __device__ __forceinline__ c32 cmul_mi(c32 a) { return {a.y, -a.x}; }
// +i * a
__host__ __device__ __forceinline__ c32 cmul_pi(c32 a) { return {-a.y, a.x}; }

// ---------------------------------------------------------------------------
// Compile-time twiddle constants W_N^m = exp(-2 pi i m / N), from a double-precision
// Taylor series on the reduced angle; quarter and eighth turns are exact.
namespace detail {
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double taylor_sin(double x) {
  double term = x, sum = x;
  for (int n = 1; n < 30; ++n) {
    term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double taylor_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 30; ++n) {
    term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    sum += term;
  }
  return sum;
}
// cos / sin of 2 pi m / N for 0 <= m < N.
constexpr double cos_frac(int m, int N) {
  return (8 * m == N)       ? 0.70710678118654752440
         : (8 * m == 3 * N) ? -0.70710678118654752440
         : (8 * m == 5 * N) ? -0.70710678118654752440
         : (8 * m == 7 * N) ? 0.70710678118654752440
                            : taylor_cos(2.0 * kPi * ((m <= N / 2) ? m : m - N) / N);
}
constexpr double sin_frac(int m, int N) {
  return (8 * m == N)       ? 0.70710678118654752440
         : (8 * m == 3 * N) ? 0.70710678118654752440
         : (8 * m == 5 * N) ? -0.70710678118654752440
         : (8 * m == 7 * N) ? -0.70710678118654752440
                            : taylor_sin(2.0 * kPi * ((m <= N / 2) ? m : m - N) / N);
}
}  // namespace detail

// a * W_N^M (forward: exp(-2 pi i M/N); INV: the conjugate).
template <int N, int M, bool INV>
__host__ __device__ __forceinline__ c32 twc(c32 a) {
  constexpr int m = ((M % N) + N) % N;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (2 * m == N) {
    return {-a.x, -a.y};
  } else if constexpr (4 * m == N) {
    return INV ? cmul_pi(a) : cmul_mi(a);
  } else if constexpr (4 * m == 3 * N) {
    return INV ? cmul_mi(a) : cmul_pi(a);
  } else {
    constexpr float c = (float)detail::cos_frac(m, N);
    constexpr float s = (float)(INV ? detail::sin_frac(m, N) : -detail::sin_frac(m, N));
    return cmul(a, c32{c, s});
  }
}

// ---------------------------------------------------------------------------
// Small DFTs, in place, natural order, unnormalised.

template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<1, INV> {
  __host__ __device__ __forceinline__ static void run(c32*) {}
};

template <bool INV>
struct Dft<2, INV> {
  __host__ __device__ __forceinline__ static void run(c32* v) {
    c32 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<3, INV> {
  __host__ __device__ __forceinline__ static void run(c32* v) {
    constexpr float h = 0.86602540378443864676f;  // sin(2 pi / 3)
    constexpr float g = INV ? -h : h;
    c32 a = v[0], t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
    c32 m = {fmaf(-0.5f, t1.x, a.x), fmaf(-0.5f, t1.y, a.y)};
    // forward: X1 = m - i h t2, X2 = m + i h t2 (the product folded into the sums)
    v[0] = cadd(a, t1);
    v[1] = c32{fmaf(g, t2.y, m.x), fmaf(-g, t2.x, m.y)};
    v[2] = c32{fmaf(-g, t2.y, m.x), fmaf(g, t2.x, m.y)};
  }
};

template <bool INV>
struct Dft<4, INV> {
  __host__ __device__ __forceinline__ static void run(c32* v) {
    c32 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    c32 t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
    c32 it3 = INV ? cmul_pi(t3) : cmul_mi(t3);
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, it3);
    v[3] = csub(t1, it3);
  }
};

template <bool INV>
struct Dft<5, INV> {
  __host__ __device__ __forceinline__ static void run(c32* v) {
    constexpr float c1 = 0.30901699437494742410f;   // cos(2 pi/5)
    constexpr float c2 = -0.80901699437494742410f;  // cos(4 pi/5)
    constexpr float s1 = 0.95105651629515357212f;   // sin(2 pi/5)
    constexpr float s2 = 0.58778525229247312917f;   // sin(4 pi/5)
    c32 a = v[0];
    c32 t1 = cadd(v[1], v[4]), t3 = csub(v[1], v[4]);
    c32 t2 = cadd(v[2], v[3]), t4 = csub(v[2], v[3]);
    c32 m1 = {fmaf(c1, t1.x, fmaf(c2, t2.x, a.x)), fmaf(c1, t1.y, fmaf(c2, t2.y, a.y))};
    c32 m2 = {fmaf(c2, t1.x, fmaf(c1, t2.x, a.x)), fmaf(c2, t1.y, fmaf(c1, t2.y, a.y))};
    c32 p1 = {fmaf(s1, t3.x, s2 * t4.x), fmaf(s1, t3.y, s2 * t4.y)};
    c32 p2 = {fmaf(s2, t3.x, -s1 * t4.x), fmaf(s2, t3.y, -s1 * t4.y)};
    // forward: X1 = m1 - i p1, X4 = m1 + i p1, X2 = m2 - i p2, X3 = m2 + i p2
    c32 q1 = INV ? cmul_pi(p1) : cmul_mi(p1);
    c32 q2 = INV ? cmul_pi(p2) : cmul_mi(p2);
    v[0] = cadd(a, cadd(t1, t2));
    v[1] = cadd(m1, q1);
    v[4] = csub(m1, q1);
    v[2] = cadd(m2, q2);
    v[3] = csub(m2, q2);
  }
};

// Composite radix R = R1 * R2: input index n = R2 n1 + n2, output k = k1 + R1 k2.
template <int R1, int R2, bool INV>
struct DftCT {
  static constexpr int R = R1 * R2;
  template <int N2>
  __host__ __device__ __forceinline__ static void inner(c32* v, c32 (&y)[R2][R1]) {
    if constexpr (N2 < R2) {
      c32 t[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) t[n1] = v[R2 * n1 + N2];
      Dft<R1, INV>::run(t);
      twiddle_row<N2, 0>(t, y[N2]);
      inner<N2 + 1>(v, y);
    }
  }
  template <int N2, int K1>
  __host__ __device__ __forceinline__ static void twiddle_row(const c32* t, c32* yrow) {
    if constexpr (K1 < R1) {
      yrow[K1] = twc<R, N2 * K1, INV>(t[K1]);
      twiddle_row<N2, K1 + 1>(t, yrow);
    }
  }
  __host__ __device__ __forceinline__ static void run(c32* v) {
    c32 y[R2][R1];
    inner<0>(v, y);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      c32 t[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) t[n2] = y[n2][k1];
      Dft<R2, INV>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = t[k2];
    }
  }
};

// Composite radix R = R1 * R2 with coprime factors, prime-factor (Good-Thomas) split:
// input n = (R2 n1 + R1 n2) mod R and output k with k = k1 (mod R1), k = k2 (mod R2)
// turn the R-point DFT into R2 DFTs of length R1 followed by R1 DFTs of length R2 with
// no twiddle factors in between.  Both index maps are compile-time register renames.
namespace detail {
constexpr int inverse_mod(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return m == 1 ? 0 : -1;
}
}  // namespace detail

template <int R1, int R2, bool INV>
struct DftPFA {
  static constexpr int R = R1 * R2;
  // k = (k1 E1 + k2 E2) mod R with E1 = 1 (mod R1), 0 (mod R2) and E2 the converse
  static constexpr int E1 = R2 * detail::inverse_mod(R2 % R1, R1);
  static constexpr int E2 = R1 * detail::inverse_mod(R1 % R2, R2);
  static_assert(E1 % R1 == 1 % R1 && E1 % R2 == 0 && E2 % R2 == 1 % R2 && E2 % R1 == 0, "factors must be coprime");
  __host__ __device__ __forceinline__ static void run(c32* v) {
    c32 y[R2][R1];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
      c32 t[R1];
#pragma unroll
      for (int n1 = 0; n1 < R1; ++n1) t[n1] = v[(R2 * n1 + R1 * n2) % R];
      Dft<R1, INV>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < R1; ++k1) y[n2][k1] = t[k1];
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      c32 t[R2];
#pragma unroll
      for (int n2 = 0; n2 < R2; ++n2) t[n2] = y[n2][k1];
      Dft<R2, INV>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[(k1 * E1 + k2 * E2) % R] = t[k2];
    }
  }
};

template <bool INV> struct Dft<6, INV> : DftPFA<2, 3, INV> {};
template <bool INV> struct Dft<8, INV> : DftCT<2, 4, INV> {};
template <bool INV> struct Dft<9, INV> : DftCT<3, 3, INV> {};
template <bool INV> struct Dft<10, INV> : DftPFA<2, 5, INV> {};
template <bool INV> struct Dft<12, INV> : DftPFA<3, 4, INV> {};
template <bool INV> struct Dft<15, INV> : DftPFA<3, 5, INV> {};
template <bool INV> struct Dft<16, INV> : DftCT<4, 4, INV> {};
template <bool INV> struct Dft<18, INV> : DftPFA<2, 9, INV> {};
template <bool INV> struct Dft<20, INV> : DftPFA<4, 5, INV> {};
template <bool INV> struct Dft<24, INV> : DftPFA<3, 8, INV> {};
template <bool INV> struct Dft<27, INV> : DftCT<3, 9, INV> {};
template <bool INV> struct Dft<30, INV> : DftPFA<5, 6, INV> {};

// ---------------------------------------------------------------------------
// Plans: a radix sequence (first pass first) whose product is the length.

template <int... Rs>
struct Radices {
  static constexpr int count = sizeof...(Rs);
  static constexpr int values[count] = {Rs...};
  static constexpr int product() { return (1 * ... * Rs); }
  static constexpr bool pfa = false;
  // Natural order in and out: position x holds element x.
  __host__ __device__ static constexpr int in_pos(int n) { return n; }
  __host__ __device__ static constexpr int out_pos(int k) { return k; }
  __host__ __device__ static constexpr int in_index(int x) { return x; }
  __host__ __device__ static constexpr int out_index(int x) { return x; }
};

namespace detail {
template <class Done, class Todo>
struct Rev;
template <int... D>
struct Rev<Radices<D...>, Radices<>> {
  using type = Radices<D...>;
};
template <int... D, int H, int... T>
struct Rev<Radices<D...>, Radices<H, T...>> {
  using type = typename Rev<Radices<H, D...>, Radices<T...>>::type;
};
}  // namespace detail

// The same factorisation with the passes in reverse order.
template <class RS>
struct ReversePlan;
template <int... Rs>
struct ReversePlan<Radices<Rs...>> {
  using type = typename detail::Rev<Radices<>, Radices<Rs...>>::type;
};
template <class RS>
using Reverse = typename ReversePlan<RS>::type;

// ---------------------------------------------------------------------------
// Prime-factor plans.  A length L = L_0 L_1 ... L_{P-1} with pairwise coprime factors
// is computed as a P-dimensional DFT with no twiddle factors at all (Good-Thomas):
// the data sit in an L_0 x L_1 x ... array, dimension 0 slowest, so that element
// (n_0, n_1, ...) is at position x = sum n_d S_d with S_d the product of the later
// factors.  The input element at (n_0, ...) is x[(sum n_d L/L_d) mod L] (the
// Ruritanian map), and after one L_d-point DFT along every dimension d the element at
// (k_0, ...) is X[k] for the k with k = k_d (mod L_d) for every d (the Chinese
// remainder map): W_L^{nk} splits into the product of W_{L_d}^{n_d k_d}.  Pass p
// transforms dimension p in place (butterfly j reads and writes x = (j / S) S L_p +
// j mod S + q S, S = S_p).  The inverse transform runs the same dimensions in reverse
// order on the same array, from the spectrum at the Chinese-remainder positions to the
// signal at the Ruritanian ones.
template <int... Ls>
struct Coprime {
  static constexpr int count = sizeof...(Ls);
  static constexpr int values[count] = {Ls...};
  static constexpr int product() { return (1 * ... * Ls); }
  static constexpr bool pfa = true;
  static constexpr int L = (1 * ... * Ls);
  __host__ __device__ static constexpr int stride(int d) {
    int s = 1;
    for (int i = d + 1; i < count; ++i) s *= values[i];
    return s;
  }
  static constexpr bool coprime() {
    for (int a = 0; a < count; ++a)
      for (int b = a + 1; b < count; ++b)
        for (int f = 2; f <= values[a]; ++f)
          if (values[a] % f == 0 && values[b] % f == 0) return false;
    return true;
  }
  static_assert(coprime(), "prime-factor plans need pairwise coprime factors");
  // Ruritanian map: the natural index of the element at position x, and its inverse.
  __host__ __device__ static constexpr int rur_index(int x) {
    long n = 0;
    for (int d = 0; d < count; ++d) n += (long)((x / stride(d)) % values[d]) * (L / values[d]);
    return (int)(n % L);
  }
  __host__ __device__ static constexpr int rur_pos(int n) {
    int x = 0;
    for (int d = 0; d < count; ++d)
      x += (int)(((long)n * detail::inverse_mod((L / values[d]) % values[d], values[d])) % values[d]) * stride(d);
    return x;
  }
  // Chinese-remainder map: the natural index of the element at position x, and its
  // inverse.
  __host__ __device__ static constexpr int crt_index(int x) {
    long k = 0;
    for (int d = 0; d < count; ++d) {
      const long e = (long)(L / values[d]) * detail::inverse_mod((L / values[d]) % values[d], values[d]);
      k += (long)((x / stride(d)) % values[d]) * e;
    }
    return (int)(k % L);
  }
  __host__ __device__ static constexpr int crt_pos(int k) {
    int x = 0;
    for (int d = 0; d < count; ++d) x += (k % values[d]) * stride(d);
    return x;
  }
  // Position of the natural index L - k (mod L) of the spectrum at position x: every
  // coordinate negated.
  __host__ __device__ static constexpr int crt_neg(int x) {
    int y = 0;
    for (int d = 0; d < count; ++d) {
      const int k = (x / stride(d)) % values[d];
      y += (k == 0 ? 0 : values[d] - k) * stride(d);
    }
    return y;
  }
  __host__ __device__ static constexpr int in_pos(int n) { return rur_pos(n); }
  __host__ __device__ static constexpr int out_pos(int k) { return crt_pos(k); }
  __host__ __device__ static constexpr int in_index(int x) { return rur_index(x); }
  __host__ __device__ static constexpr int out_index(int x) { return crt_index(x); }
};

// The inverse-direction plan of a prime-factor plan: dimensions in reverse order on the
// same array, spectrum in at the Chinese-remainder positions, signal out at the
// Ruritanian ones.
template <class CP>
struct CoprimeRev {
  using Fwd = CP;
  static constexpr int count = CP::count;
  static constexpr int product() { return CP::product(); }
  static constexpr bool pfa = true;
  __host__ __device__ static constexpr int in_pos(int k) { return CP::crt_pos(k); }
  __host__ __device__ static constexpr int out_pos(int n) { return CP::rur_pos(n); }
  __host__ __device__ static constexpr int in_index(int x) { return CP::crt_index(x); }
  __host__ __device__ static constexpr int out_index(int x) { return CP::rur_index(x); }
};
template <int... Ls>
struct ReversePlan<Coprime<Ls...>> {
  using type = CoprimeRev<Coprime<Ls...>>;
};

// Offset of pass p's twiddles in the packed table of a plan: the sum over earlier
// passes of Ns (r - 1), Ns = product of the earlier radices.
template <class RS>
constexpr int tw_offset(int p) {
  int off = 0, ns = 1;
  for (int i = 0; i < p; ++i) {
    off += ns * (RS::values[i] - 1);
    ns *= RS::values[i];
  }
  return off;
}
template <class RS>
constexpr int span_before(int p) {
  int ns = 1;
  for (int i = 0; i < p; ++i) ns *= RS::values[i];
  return ns;
}
template <class RS>
constexpr int tw_size() {
  return tw_offset<RS>(RS::count);
}

// LDS slot of logical element x of a batch of B interleaved transforms.  The plans
// keep the strided accesses of every pass free of bank conflicts (odd first-pass
// strides for single transforms, 64-byte runs for interleaved batches), so elements are
// stored unpadded and every in-pass offset is a compile-time constant.
template <int B>
__host__ __device__ constexpr int lds_slot(int x) {
  return x;
}
template <int B>
__host__ __device__ constexpr int lds_size(int n) {
  return lds_slot<B>(n - 1) + 1;
}

// Twiddle-table entry i: on the device a global-memory load (scalar base + 32-bit
// vector offset, not a flat access); in the host emulator a plain load.
__host__ __device__ __forceinline__ c32 tw_load(const c32* tw, int i) {
#if defined(__HIP_DEVICE_COMPILE__)
  const __attribute__((address_space(1))) float* p = (const __attribute__((address_space(1))) float*)tw;
  return c32{p[2 * i], p[2 * i + 1]};
#else
  return tw[i];
#endif
}

// Pass P of plan RS on a batch of B interleaved transforms processed by T threads.
// Butterfly g = tid + round * T (round < ROUNDS, g < TOT) works on transform b = g mod B,
// butterfly j = g / B: it reads elements j + q NB (q < R), multiplies by the twiddles
// W_{Ns R}^{k q} (k = j mod Ns), applies the radix-R DFT and writes element
// (j - k) R + k + q Ns.  Element i of transform b lives at LDS slot lds_slot<B>(i B + b).
template <class RS, int P, int B, int T>
struct Pass {
  static constexpr int L = RS::product();
  static constexpr int R = RS::values[P];
  static constexpr int NS = span_before<RS>(P);
  static constexpr int NB = L / R;
  static constexpr int TOT = NB * B;
  static constexpr int ROUNDS = (TOT + T - 1) / T;
  static constexpr int TWOFF = tw_offset<RS>(P);
  // whether butterfly j writes exactly the elements it reads (then a thread's stores
  // never overwrite what another thread of the same pass has yet to load): not in a
  // Stockham pass
  static constexpr bool in_place = false;
  __host__ __device__ static constexpr bool full() { return TOT % T == 0; }
  __host__ __device__ __forceinline__ static int in_el(int j, int q) { return j + q * NB; }
  __host__ __device__ __forceinline__ static int out_el(int j, int q) {
    const int k = j % NS;
    return (j - k) * R + k + q * NS;
  }
  // Twiddle and DFT in registers; tw is the plan's packed forward table.  Radices 5 to
  // 16 read four table entries per butterfly and form the other twiddles in registers
  // (butterfly_pow4): the kernels' vector-memory paths are busier than their VALUs.
  template <bool INV>
  __host__ __device__ __forceinline__ static void butterfly(c32* v, int j, const c32* tw) {
    if constexpr (NS > 1 && R >= 5 && R <= 16) {
      butterfly_pow4<INV>(v, j, tw);
      return;
    }
    if constexpr (NS > 1) {
      const int t = TWOFF + (j % NS) * (R - 1);
#pragma unroll
      for (int q = 1; q < R; ++q) {
        const c32 w = tw_load(tw, t + q - 1);
        v[q] = INV ? cmulc(v[q], w) : cmul(v[q], w);
      }
    }
    Dft<R, INV>::run(v);
  }
  // The same reading only W^k .. W^4k (W = W_{Ns R}, k = j mod Ns) from the table and
  // forming the higher powers as complex products of those (W^8k = (W^4k)^2,
  // W^12k = W^8k W^4k, W^(m+r)k = W^mk W^rk): four table entries instead of R - 1, for
  // R - 5 more complex products (R <= 16).
  template <bool INV>
  __host__ __device__ __forceinline__ static void butterfly_pow4(c32* v, int j, const c32* tw) {
    static_assert(R <= 16, "powers up to W^15k");
    if constexpr (NS > 1) {
      const int t = TWOFF + (j % NS) * (R - 1);
      c32 p[R];
#pragma unroll
      for (int q = 1; q < R && q <= 4; ++q) p[q] = tw_load(tw, t + q - 1);
      c32 p8 = {1.f, 0.f}, p12 = {1.f, 0.f};
      if constexpr (R > 8) p8 = cmul(p[4], p[4]);
      if constexpr (R > 12) p12 = cmul(p8, p[4]);
#pragma unroll
      for (int q = 5; q < R; ++q) {
        if (q == 8) p[q] = p8;
        else if (q == 12) p[q] = p12;
        else p[q] = cmul(q < 8 ? p[4] : (q < 12 ? p8 : p12), p[q & 3]);
      }
#pragma unroll
      for (int q = 1; q < R; ++q) v[q] = INV ? cmulc(v[q], p[q]) : cmul(v[q], p[q]);
    }
    Dft<R, INV>::run(v);
  }
  // The same with this pass's twiddles in a table of its own (entry k (R - 1) + q - 1 =
  // W_{Ns R}^{k q}), e.g. a copy in LDS.
  template <bool INV>
  __host__ __device__ __forceinline__ static void butterfly_own(c32* v, int j, const c32* twp) {
    if constexpr (NS > 1) {
      const int t = (j % NS) * (R - 1);
#pragma unroll
      for (int q = 1; q < R; ++q) {
        const c32 w = twp[t + q - 1];
        v[q] = INV ? cmulc(v[q], w) : cmul(v[q], w);
      }
    }
    Dft<R, INV>::run(v);
  }
};

// Pass P of a prime-factor plan: the L_P-point DFT along dimension P, in place, with no
// twiddles.  NS is the dimension's stride and NB = L / L_P the butterflies per
// transform, so that as in a Stockham pass out_el(j, q) = out_el(j, 0) + q NS, and
// pass 0 reads elements j + q NB.
template <int... Ls, int P, int B, int T>
struct Pass<Coprime<Ls...>, P, B, T> {
  using CP = Coprime<Ls...>;
  static constexpr int L = CP::L;
  static constexpr int R = CP::values[P];
  static constexpr int NS = CP::stride(P);
  static constexpr int NB = L / R;
  static constexpr int TOT = NB * B;
  static constexpr int ROUNDS = (TOT + T - 1) / T;
  static constexpr int TWOFF = 0;
  static constexpr bool in_place = true;  // out_el = in_el: each dimension in place
  __host__ __device__ static constexpr bool full() { return TOT % T == 0; }
  __host__ __device__ __forceinline__ static int in_el(int j, int q) {
    if constexpr (NS == NB)
      return j + q * NS;  // dimension 0: j < NB = NS
    else if constexpr (NS == 1)
      return j * R + q;
    else
      return (j / NS) * NS * R + j % NS + q * NS;
  }
  __host__ __device__ __forceinline__ static int out_el(int j, int q) { return in_el(j, q); }
  template <bool INV>
  __host__ __device__ __forceinline__ static void butterfly(c32* v, int, const c32*) {
    Dft<R, INV>::run(v);
  }
};
template <class CP, int P, int B, int T>
struct Pass<CoprimeRev<CP>, P, B, T> : Pass<CP, CP::count - 1 - P, B, T> {};

}  // namespace prnu
