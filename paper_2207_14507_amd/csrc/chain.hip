// Device-side candidate generation, per-frame argmax and the warm-start chain of
// Algorithm 1 (Sec. 3.2): see chain.hpp for how the kernels surround a launch of the
// search kernels.
#include <math.h>

#include "chain.hpp"

namespace prnu {

namespace {

// Grid nodes in FP64, generated exactly as centre + (k - (n - 1) / 2) * step with every
// product and sum rounded on its own (no fused multiply-add), the form the host-side
// grid helpers use, so that the device and the host name the same candidates.
#pragma clang fp contract(off)
__device__ double grid_node_d(int k, int n, double lo, double hi) {
  const double centre = (lo + hi) / 2.0;
  const double step = n > 1 ? (hi - lo) / (double)(n - 1) : 0.0;
  const double half = (double)(n - 1) / 2.0;
  return centre + ((double)k - half) * step;
}

__device__ double local_node_d(int k, int n, double centre, double step) {
  const double half = (double)(n - 1) / 2.0;
  return centre + ((double)k - half) * step;
}

// Inverse-warp coefficients of a candidate (Eq. 4, similarity form):
// a = cos(theta) / s, b = sin(theta) / s in FP64, rounded once to float.
__device__ CandParam param_of(const CandSite& c, int slot, int fslot) {
  const double th = c.t * (3.14159265358979323846 / 180.0);
  double sn, cs;
  sincos(th, &sn, &cs);
  CandParam p;
  p.a = (float)(cs / c.s);
  p.b = (float)(sn / c.s);
  p.frame = slot;
  p.fp = fslot;
  return p;
}
#pragma clang fp contract(on)

__device__ CandSite gen_site(const GridGen& g, int i) {
  if (g.kind == kGenList) return g.list[i];
  const int si = i / g.nr, ri = i % g.nr;
  if (g.kind == kGenFull) return CandSite{grid_node_d(si, g.ns, g.lo0, g.hi0), grid_node_d(ri, g.nr, g.lo1, g.hi1)};
  const ChainState c = *g.centre;
  return CandSite{local_node_d(si, g.ns, c.cs, g.lo0), local_node_d(ri, g.nr, c.ct, g.lo1)};
}

__global__ __launch_bounds__(256) void k_gen(const ItemDesc* items, CandParam* cand, CandSite* site) {
  const ItemDesc& it = items[blockIdx.x];
  const int i = (int)blockIdx.y * 256 + (int)threadIdx.x;
  if (i >= it.n) return;
  const CandSite c = gen_site(it.gen, i);
  cand[it.off + i] = param_of(c, it.slot, it.fslot);
  site[it.off + i] = c;
}

// x beats the current best (bv, bi): finite comparison in FP64, the lower index on
// equal scores, NaN never.
__device__ __forceinline__ bool beats(double v, int i, double bv, int bi) {
  if (v != v) return false;
  return bi < 0 || v > bv || (v == bv && i < bi);
}

// Best of records [0, n) (index -1 if every score is NaN), valid in thread 0.
template <int T>
__device__ void segment_best(const CandRecord* rec, int n, double& bv, int& bi) {
  __shared__ double sv[T / 64];
  __shared__ int si[T / 64];
  bv = 0.0;
  bi = -1;
  for (int i = (int)threadIdx.x; i < n; i += T) {
    const double v = rec[i].pce;
    if (beats(v, i, bv, bi)) {
      bv = v;
      bi = i;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(bv, o, 64);
    const int oi = __shfl_xor(bi, o, 64);
    if (oi >= 0 && beats(ov, oi, bv, bi)) {
      bv = ov;
      bi = oi;
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sv[w] = bv;
    si[w] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < T / 64; ++k)
      if (si[k] >= 0 && beats(sv[k], si[k], bv, bi)) {
        bv = sv[k];
        bi = si[k];
      }
  }
}

// Fold segment best (record r at list position idx, or none when idx < 0) into the
// running best; candidates of earlier segments win ties.
__device__ void fold(FrameBest& fb, const CandRecord* rec, const CandSite* site, int bi, int base, int n) {
  if (bi >= 0) {
    const double v = rec[bi].pce;
    if (fb.index < 0 || v > fb.rec.pce) {
      fb.rec = rec[bi];
      fb.s = site[bi].s;
      fb.t = site[bi].t;
      fb.index = base + bi;
    }
  }
  fb.n_eval = base + n;
}

// The frame's result record and the centre of the video's next local grid.
__device__ void commit(const ItemDesc& it, const FrameBest& fb) {
  prnu_frame_result r;
  r.pce = 0.0;
  r.rho = 0.0;
  r.scale = 0.0;
  r.rot_deg = 0.0;
  r.dx = r.dy = 0;
  r.cand_index = 0;
  r.fell_back = fb.fell_back;
  r.n_evaluated = fb.n_eval;
  r.iterations = it.mode == kModeRefine ? it.iter : 0;
  r.used_init = 0;
  if (fb.index < 0) {
    r.status = PRNU_E_NONFINITE;
    r.pce = __builtin_nan("");
  } else {
    r.pce = fb.rec.pce;
    r.rho = fb.rec.rho;
    r.scale = fb.s;
    r.rot_deg = fb.t;
    r.dx = fb.rec.dx;
    r.dy = fb.rec.dy;
    r.cand_index = fb.index;
    r.status = isfinite(fb.rec.pce) ? PRNU_OK : PRNU_E_NONFINITE;
    if (it.state) {
      it.state->cs = fb.s;
      it.state->ct = fb.t;
      it.state->have = 1;
    }
  }
  if (it.result) *it.result = r;
}

// Start phase: one block per item over its segment of the launch's list.  Merge phase:
// one block per warm item whose fallback grid was searched, over its fallback segment.
template <int T>
__global__ __launch_bounds__(T) void k_argmax(const ItemDesc* items, ItemOut* outs, const CandRecord* rec,
                                              const CandSite* site, int merge_fallback, const CandRecord* fb_rec,
                                              const CandSite* fb_site) {
  const ItemDesc& it = items[blockIdx.x];
  ItemOut& out = outs[blockIdx.x];
  double bv;
  int bi;
  if (merge_fallback) {
    if (it.mode != kModeWarm || !out.need) return;  // uniform per block
    const CandRecord* r = fb_rec + out.fb_off;
    const CandSite* c = fb_site + out.fb_off;
    segment_best<T>(r, it.fb_n, bv, bi);
    if (threadIdx.x == 0) {
      FrameBest fb = *it.best;
      fold(fb, r, c, bi, fb.n_eval, it.fb_n);
      *it.best = fb;
      commit(it, fb);
    }
    return;
  }
  const CandRecord* r = rec + it.off;
  const CandSite* c = site + it.off;
  segment_best<T>(r, it.n, bv, bi);
  if (threadIdx.x != 0) return;
  FrameBest fb;
  if (it.mode == kModeRefine && it.merge) {
    fb = *it.best;
  } else {
    fb.index = -1;
    fb.n_eval = 0;
    fb.fell_back = 0;
    fb.pad = 0;
    fb.s = fb.t = 0.0;
    fb.rec = CandRecord{};
  }
  fold(fb, r, c, bi, fb.n_eval, it.n);
  out.need = 0;
  out.fb_off = 0;
  out.seg_index = bi;
  out.seg_s = bi >= 0 ? c[bi].s : 0.0;
  out.seg_t = bi >= 0 ? c[bi].t : 0.0;
  out.seg_pce = bi >= 0 ? r[bi].pce : 0.0;
  if (it.mode == kModeWarm) {
    if (!it.state->have) {
      // no earlier frame of the video has a finite result: this frame is searched like
      // a first frame, on the full grid alone (the local segment does not count)
      fb.index = -1;
      fb.n_eval = 0;
      fb.fell_back = 0;
      out.need = 1;
    } else {
      // the local best falls short (or nothing finite was scored): the full grid follows
      out.need = (bi < 0 || !(r[bi].pce >= it.fallback_pce)) ? 1 : 0;
      fb.fell_back = out.need;
    }
  }
  *it.best = fb;
  if (it.mode != kModeWarm || !out.need) commit(it, fb);
}

__global__ void k_plan(const ItemDesc* items, int n, ItemOut* outs, int* n_dev) {
  if (threadIdx.x != 0) return;
  int total = 0;
  for (int i = 0; i < n; ++i) {
    const bool need = items[i].mode == kModeWarm && outs[i].need;
    outs[i].fb_off = total;
    if (need) total += items[i].fb_n;
  }
  *n_dev = total;
}

__global__ __launch_bounds__(256) void k_fill(const ItemDesc* items, int n, const ItemOut* outs, const int* n_dev,
                                              CandParam* fb_cand, CandSite* fb_site) {
  const int e = (int)blockIdx.x * 256 + (int)threadIdx.x;
  if (e >= *n_dev) return;
  for (int i = 0; i < n; ++i) {
    const ItemDesc& it = items[i];
    if (it.mode != kModeWarm || !outs[i].need) continue;
    const int j = e - outs[i].fb_off;
    if (j < 0 || j >= it.fb_n) continue;
    const CandSite c = gen_site(it.full, j);
    fb_cand[e] = param_of(c, it.slot, it.fslot);
    fb_site[e] = c;
    return;
  }
}

__global__ void k_chain_init(ChainState* st, int has_init, double cs, double ct) {
  st->cs = cs;
  st->ct = ct;
  st->have = has_init;
  st->pad = 0;
}

__global__ void k_put(Blob blob, unsigned char* dst) {
  for (int i = (int)threadIdx.x; i < blob.n; i += (int)blockDim.x) dst[i] = blob.b[i];
}

__global__ void k_scatter(const CandRecord* rec, int n, double* pce, double* rho, int32_t* dx, int32_t* dy) {
  const int i = (int)blockIdx.x * 256 + (int)threadIdx.x;
  if (i >= n) return;
  const CandRecord r = rec[i];
  if (pce) pce[i] = r.pce;
  if (rho) rho[i] = r.rho;
  if (dx) dx[i] = r.dx;
  if (dy) dy[i] = r.dy;
}

}  // namespace

hipError_t launch_gen(const ItemDesc* items, int n, int max_n, CandParam* cand, CandSite* site, hipStream_t s) {
  if (n <= 0 || max_n <= 0) return hipSuccess;
  k_gen<<<dim3((unsigned)n, (unsigned)((max_n + 255) / 256)), 256, 0, s>>>(items, cand, site);
  return hipGetLastError();
}

hipError_t launch_argmax(const ItemDesc* items, int n, ItemOut* outs, const CandRecord* rec, const CandSite* site,
                         bool merge_fallback, const CandRecord* fb_rec, const CandSite* fb_site, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_argmax<256><<<dim3((unsigned)n), 256, 0, s>>>(items, outs, rec, site, merge_fallback ? 1 : 0, fb_rec, fb_site);
  return hipGetLastError();
}

hipError_t launch_plan(const ItemDesc* items, int n, ItemOut* outs, int* n_dev, hipStream_t s) {
  k_plan<<<1, 64, 0, s>>>(items, n, outs, n_dev);
  return hipGetLastError();
}

hipError_t launch_fill(const ItemDesc* items, int n, const ItemOut* outs, const int* n_dev, int max_fb,
                       CandParam* fb_cand, CandSite* fb_site, hipStream_t s) {
  if (max_fb <= 0) return hipSuccess;
  k_fill<<<dim3((unsigned)((max_fb + 255) / 256)), 256, 0, s>>>(items, n, outs, n_dev, fb_cand, fb_site);
  return hipGetLastError();
}

hipError_t launch_chain_init(ChainState* st, int has_init, double cs, double ct, hipStream_t s) {
  k_chain_init<<<1, 1, 0, s>>>(st, has_init, cs, ct);
  return hipGetLastError();
}

hipError_t launch_put(const Blob& blob, void* dst, hipStream_t s) {
  if (blob.n <= 0) return hipSuccess;
  k_put<<<1, 256, 0, s>>>(blob, reinterpret_cast<unsigned char*>(dst));
  return hipGetLastError();
}

hipError_t launch_scatter(const CandRecord* rec, int n, double* pce, double* rho, int32_t* dx, int32_t* dy,
                          hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_scatter<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(rec, n, pce, rho, dx, dy);
  return hipGetLastError();
}

}  // namespace prnu
