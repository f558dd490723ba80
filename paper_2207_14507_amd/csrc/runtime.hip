// Host runtime behind prnu.h: context, device-resident fingerprints, grid
// descriptions, chunked launch of the search kernels with the device-side argmax and
// warm-start chain around them (chain.hip), and the synchronous searches.  The serving
// engine (submit / poll) lives in serving.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "fft_exec.hpp"
#include "runtime.hpp"

namespace prnu {

thread_local std::string g_last_error;

prnu_status fail(prnu_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

prnu_status Context::hip_fail(hipError_t e, const char* what) {
  failed = true;
  return fail(PRNU_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// Buffers.

hipError_t DevBuf::reserve(size_t n) {
  if (n <= cap) return hipSuccess;
  release();
  hipError_t e = hipMalloc(&ptr, n);
  if (e != hipSuccess) {
    ptr = nullptr;
    return e;
  }
  cap = n;
  return hipSuccess;
}

void DevBuf::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  cap = 0;
}

hipError_t HostBuf::reserve(size_t n) {
  if (n <= cap) return hipSuccess;
  release();
  hipError_t e = hipHostMalloc(&ptr, n, hipHostMallocDefault);
  if (e != hipSuccess) {
    ptr = nullptr;
    return e;
  }
  cap = n;
  return hipSuccess;
}

void HostBuf::release() {
  if (ptr) (void)hipHostFree(ptr);
  ptr = nullptr;
  cap = 0;
}

// ---------------------------------------------------------------------------
// Grids (FP64, generated exactly as centre + (k - (n-1)/2) * step).

#pragma clang fp contract(off)
double grid_node(int k, int n, double lo, double hi) {
  const double centre = (lo + hi) / 2.0;
  const double step = n > 1 ? (hi - lo) / (double)(n - 1) : 0.0;
  const double half = (double)(n - 1) / 2.0;
  return centre + ((double)k - half) * step;
}

double local_node(int k, int n, double centre, double step) {
  const double half = (double)(n - 1) / 2.0;
  return centre + ((double)k - half) * step;
}

void full_candidates(const prnu_grid& g, std::vector<Cand>& out) {
  out.clear();
  for (int i = 0; i < g.n_scale; ++i)
    for (int j = 0; j < g.n_rot; ++j)
      out.push_back(Cand{grid_node(i, g.n_scale, g.scale_lo, g.scale_hi), grid_node(j, g.n_rot, g.rot_lo_deg, g.rot_hi_deg)});
}

void local_candidates(const prnu_search_opts& o, double cs, double ct, std::vector<Cand>& out) {
  out.clear();
  for (int i = 0; i < o.local_n_scale; ++i)
    for (int j = 0; j < o.local_n_rot; ++j)
      out.push_back(Cand{local_node(i, o.local_n_scale, cs, o.local_dscale), local_node(j, o.local_n_rot, ct, o.local_drot_deg)});
}

// Inverse-warp coefficients of a candidate: a = cos(theta)/s, b = sin(theta)/s in FP64,
// rounded once to float.
CandParam make_param(const Cand& c, int frame, int fp) {
  const double th = c.rot_deg * (3.14159265358979323846 / 180.0);
  CandParam p;
  p.a = (float)(std::cos(th) / c.scale);
  p.b = (float)(std::sin(th) / c.scale);
  p.frame = frame;
  p.fp = fp;
  return p;
}
#pragma clang fp contract(on)

prnu_status check_shape(int M, int N, int radius) {
  if (M <= 0 || N <= 0) return fail(PRNU_E_SHAPE, "image size %dx%d must be positive", M, N);
  if (N % 2) return fail(PRNU_E_SHAPE, "width %d must be even", N);
  if (!length_supported(N)) return fail(PRNU_E_SHAPE, "width %d is not a supported transform length", N);
  if (!col_length_supported(M)) return fail(PRNU_E_SHAPE, "height %d is not a supported transform length", M);
  if (radius < 0) return fail(PRNU_E_ARG, "shift radius %d must be >= 0", radius);
  if (M < 2 * radius + 11 || N < 2 * radius + 11)
    return fail(PRNU_E_SHAPE, "image %dx%d is smaller than 2*radius+11 = %d", M, N, 2 * radius + 11);
  return PRNU_OK;
}

prnu_status validate_opts(const prnu_search_opts* o) {
  if (!o) return fail(PRNU_E_ARG, "null options");
  if (o->exclusion != 11) return fail(PRNU_E_ARG, "exclusion must be 11 (Eq. 3), got %d", o->exclusion);
  if (o->full.n_scale < 1 || o->full.n_rot < 1) return fail(PRNU_E_ARG, "empty full grid");
  if ((long)o->full.n_scale * o->full.n_rot > (1L << 20)) return fail(PRNU_E_ARG, "grid too large");
  auto scale_ok = [](double s) { return std::isfinite(s) && s >= 0.25 && s <= 4.0; };
  if (!scale_ok(o->full.scale_lo) || !scale_ok(o->full.scale_hi)) return fail(PRNU_E_ARG, "scale range must lie in [0.25, 4]");
  if (!std::isfinite(o->full.rot_lo_deg) || !std::isfinite(o->full.rot_hi_deg)) return fail(PRNU_E_ARG, "rotation range not finite");
  if (o->warm) {
    if (o->local_n_scale < 1 || o->local_n_rot < 1) return fail(PRNU_E_ARG, "empty local grid");
    if ((long)o->local_n_scale * o->local_n_rot > (1L << 20)) return fail(PRNU_E_ARG, "local grid too large");
    if (!std::isfinite(o->local_dscale) || !std::isfinite(o->local_drot_deg)) return fail(PRNU_E_ARG, "local steps");
    if (o->has_init && !scale_ok(o->init_scale)) return fail(PRNU_E_ARG, "init scale");
    if (std::fabs(o->local_dscale) * (o->local_n_scale - 1) > 1.0) return fail(PRNU_E_ARG, "local scale span too wide");
  }
  if (o->refine) {
    if (o->warm) return fail(PRNU_E_ARG, "refine and warm are exclusive");
    if (o->refine_half < 0 || o->refine_half > 50) return fail(PRNU_E_ARG, "refine_half must lie in [0, 50]");
    if (o->refine_max_iter < 1 || o->refine_max_iter > 8) return fail(PRNU_E_ARG, "refine_max_iter must lie in [1, 8]");
    if (!(o->refine_scale_step > 0.0) || !(o->refine_rot_step > 0.0) || !std::isfinite(o->refine_scale_step) ||
        !std::isfinite(o->refine_rot_step))
      return fail(PRNU_E_ARG, "refine steps must be positive");
    if (!std::isfinite(o->refine_rot_lo_deg) || !std::isfinite(o->refine_rot_hi_deg) ||
        !(o->refine_rot_hi_deg >= o->refine_rot_lo_deg))
      return fail(PRNU_E_ARG, "refine rotation range");
    const double nr = std::round((o->refine_rot_hi_deg - o->refine_rot_lo_deg) / o->refine_rot_step) + 1.0;
    if (nr > 100001.0 || nr * (2.0 * o->refine_half + 1.0) > (double)(1 << 20))
      return fail(PRNU_E_ARG, "refinement grid too large");
    const double s0 = o->has_init ? o->init_scale : 1.0;
    if (!scale_ok(s0) || o->refine_scale_step * o->refine_half >= 0.5 * s0)
      return fail(PRNU_E_ARG, "refinement scale span leaves [0.25, 4]");
  }
  return PRNU_OK;
}

// The grid of refinement iteration n (1-based) around (cs, ct): scale-major, the first
// iteration on the dense absolute rotation grid (see prnu_search_opts).
void refine_candidates(const prnu_search_opts& o, int n, double cs, double ct, std::vector<Cand>& out) {
  out.clear();
  const double f = std::pow(10.0, -(double)(n - 1));
  const int ns = 2 * o.refine_half + 1;
  const int nr = n == 1 ? (int)std::lround((o.refine_rot_hi_deg - o.refine_rot_lo_deg) / o.refine_rot_step) + 1 : ns;
  for (int i = 0; i < ns; ++i) {
    const double s = local_node(i, ns, cs, o.refine_scale_step * f);
    for (int j = 0; j < nr; ++j)
      out.push_back(Cand{s, n == 1 ? grid_node(j, nr, o.refine_rot_lo_deg, o.refine_rot_hi_deg)
                                   : local_node(j, nr, ct, o.refine_rot_step * f)});
  }
}

prnu_status validate_frames(const prnu_frames* fr, const Fingerprint& fp, int radius) {
  if (!fr) return fail(PRNU_E_ARG, "null frames");
  if (fr->n_frames < 0) return fail(PRNU_E_ARG, "negative frame count");
  if (fr->n_frames > 0 && !fr->data) return fail(PRNU_E_ARG, "null frame data");
  if (fr->dtype != PRNU_F32 && fr->dtype != PRNU_BF16) return fail(PRNU_E_ARG, "unknown dtype %d", (int)fr->dtype);
  if (fr->dtype == PRNU_BF16 && fr->n_frames > 0 && !fr->frame_scale) return fail(PRNU_E_ARG, "bf16 frames need frame_scale");
  prnu_status st = check_shape(fp.M, fp.N, radius);
  if (st != PRNU_OK) return st;
  // A frame smaller than the fingerprint is zero-padded to its size; a larger one is
  // not accepted.  The frame must hold the stored window's 2R + 11 rows and columns.
  if (fr->height > fp.M || fr->width > fp.N)
    return fail(PRNU_E_SHAPE, "frame %dx%d is larger than fingerprint %dx%d", fr->height, fr->width, fp.M, fp.N);
  if (fr->height < 2 * radius + 11 || fr->width < 2 * radius + 11)
    return fail(PRNU_E_SHAPE, "frame %dx%d is smaller than 2*radius+11 = %d", fr->height, fr->width, 2 * radius + 11);
  if (fr->row_stride < fr->width) return fail(PRNU_E_ARG, "row stride %lld < width", (long long)fr->row_stride);
  if (fr->n_frames > 1 && fr->frame_stride < fr->row_stride * fr->height) return fail(PRNU_E_ARG, "frame stride too small");
  return PRNU_OK;
}

Shape search_shape(const Fingerprint& fp, const prnu_frames* fr, int radius) {
  Shape sh{fp.M, fp.N, radius};
  sh.ey = fp.M - fr->height;
  sh.ex = fp.N - fr->width;
  return sh;
}

GridGen full_gen(const prnu_grid& g) {
  GridGen x{};
  x.kind = kGenFull;
  x.ns = g.n_scale;
  x.nr = g.n_rot;
  x.lo0 = g.scale_lo;
  x.hi0 = g.scale_hi;
  x.lo1 = g.rot_lo_deg;
  x.hi1 = g.rot_hi_deg;
  return x;
}

GridGen local_gen(const prnu_search_opts& o, const ChainState* centre) {
  GridGen x{};
  x.kind = kGenLocal;
  x.ns = o.local_n_scale;
  x.nr = o.local_n_rot;
  x.lo0 = o.local_dscale;
  x.lo1 = o.local_drot_deg;
  x.centre = centre;
  return x;
}

// ---------------------------------------------------------------------------
// Runner.

Runner::~Runner() {
  for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  for (GraphEntry& g : graphs) (void)hipGraphExecDestroy(g.exec);
}

void Runner::drop_graphs() {
  if (graphs.empty()) return;
  (void)hipStreamSynchronize(stream);
  for (GraphEntry& g : graphs) (void)hipGraphExecDestroy(g.exec);
  graphs.clear();
}

// Default FFT batch: as many candidates as the forward intermediate of batch_bytes holds.
int Runner::batch_size(const Shape& sh) const {
  if (batch_override > 0) return batch_override;
  const double per = (double)sh.M * sh.Nh() * sizeof(c32);
  const int b = (int)std::floor(batch_bytes / per);
  return std::max(1, std::min(256, b));
}

size_t Runner::workspace_bytes(const Shape& sh, int nc) const {
  return (size_t)nc * ((size_t)sh.M * tiled_cols(sh) * sizeof(c32) + (size_t)sh.band_rows() * sh.Nh() * sizeof(c32) +
                       (size_t)sh.band_rows() * sh.win_cols() * sizeof(float) +
                       (size_t)sh.row_pairs() * sizeof(double2) + (size_t)col_blocks(sh) * sizeof(double));
}

prnu_status Runner::ensure_workspace(const Shape& sh, int nc) {
  hipError_t e;
  const bool grow = (size_t)nc * sh.M * tiled_cols(sh) * sizeof(c32) > ws_inter.cap ||
                    (size_t)nc * sh.band_rows() * sh.Nh() * sizeof(c32) > ws_band.cap ||
                    (size_t)nc * sh.band_rows() * sh.win_cols() * sizeof(float) > ws_win.cap ||
                    (size_t)nc * sh.row_pairs() * sizeof(double2) > ws_norm.cap ||
                    (size_t)nc * col_blocks(sh) * sizeof(double) > ws_energy.cap;
  // Launches already queued on this stream may still use the buffers about to be
  // replaced: let them finish first.
  if (grow && (e = hipStreamSynchronize(stream)) != hipSuccess)
    return fail(PRNU_E_DEVICE, "workspace: %s", hipGetErrorString(e));
  if ((e = ws_inter.reserve((size_t)nc * sh.M * tiled_cols(sh) * sizeof(c32))) != hipSuccess ||
      (e = ws_band.reserve((size_t)nc * sh.band_rows() * sh.Nh() * sizeof(c32))) != hipSuccess ||
      (e = ws_win.reserve((size_t)nc * sh.band_rows() * sh.win_cols() * sizeof(float))) != hipSuccess ||
      (e = ws_norm.reserve((size_t)nc * sh.row_pairs() * sizeof(double2))) != hipSuccess ||
      (e = ws_energy.reserve((size_t)nc * col_blocks(sh) * sizeof(double))) != hipSuccess)
    return fail(PRNU_E_NOMEM, "workspace: %s", hipGetErrorString(e));
  return PRNU_OK;
}

static Batch make_batch(const Runner& r, const Shape& sh, int dtype, const FrameRef* frames, const FpRef* fps,
                        const CandParam* cand, const float* proj, CandRecord* rec, int start, int nc, int order,
                        const c32* twM, const c32* twMi, const c32* twN) {
  Batch b{};
  b.shape = sh;
  b.nc = nc;
  b.cand = cand + start;
  b.dtype = dtype;
  b.frames = frames;
  b.fps = fps;
  b.inter = reinterpret_cast<c32*>(r.ws_inter.ptr);
  b.band = reinterpret_cast<c32*>(r.ws_band.ptr);
  b.win = reinterpret_cast<float*>(r.ws_win.ptr);
  b.norm_part = reinterpret_cast<double2*>(r.ws_norm.ptr);
  b.energy_part = reinterpret_cast<double*>(r.ws_energy.ptr);
  b.rec = rec + start;
  b.twM = twM;
  b.twMi = twMi;
  b.twN = twN;
  b.order = order;
  b.proj = proj ? proj + (size_t)start * 9 : nullptr;
  return b;
}

hipError_t Runner::launch_all(const Shape& sh, int dtype, const FrameRef* frames, const FpRef* fps,
                              const CandParam* cand, const float* proj, CandRecord* rec, int n, const Schedule& sc,
                              const c32* twM, const c32* twMi, const c32* twN) {
  for (int start = 0; start < n; start += sc.chunk) {
    const int nc = std::min(sc.chunk, n - start);
    const Batch b = make_batch(*this, sh, dtype, frames, fps, cand, proj, rec, start, nc, sc.order, twM, twMi, twN);
    hipError_t e;
    if ((e = launch_warp_rowfft(b, stream)) != hipSuccess || (e = launch_col_product(b, stream)) != hipSuccess ||
        (e = launch_band_rowifft(b, stream)) != hipSuccess || (e = launch_pce(b, stream)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

prnu_status Runner::run(Context& ctx, const Shape& sh, int dtype, const FrameRef* frames, const FpRef* fps,
                        const CandParam* cand, CandRecord* rec, int n, const float* proj) {
  Schedule sc;
  prnu_status st = ctx.schedule(sh, dtype, *this, sc);
  if (st != PRNU_OK) return st;
  if (batch_override > 0) sc.chunk = batch_override;
  const int bc = sc.chunk;
  st = ensure_workspace(sh, std::min(bc, std::max(n, 1)));
  if (st != PRNU_OK) return st;
  const c32* twM = ctx.twiddles(kColPlan, sh.M);
  const c32* twMi = ctx.twiddles(kColPlanRev, sh.M);
  const c32* twN = ctx.twiddles(kRowPlan, sh.N);
  if (!twM || !twMi || !twN) return ctx.hip_fail(hipErrorOutOfMemory, "twiddle tables");
  if (n <= 0) return PRNU_OK;
  if (ctx.inject(ctx.fault_launch, ctx.n_launch)) return ctx.hip_fail(hipErrorLaunchFailure, "injected launch fault");
  hipError_t e;
  if (!prof_on) {
    if (!use_graphs) {
      if ((e = launch_all(sh, dtype, frames, fps, cand, proj, rec, n, sc, twM, twMi, twN)) != hipSuccess)
        return ctx.hip_fail(e, "search launch");
      return PRNU_OK;
    }
    // Replay the launch set if this exact one (shape, count, schedule, buffers) was
    // captured before; otherwise capture it now.
    const std::vector<uintptr_t> key = {
        (uintptr_t)sh.M,          (uintptr_t)sh.N,          (uintptr_t)sh.radius,      (uintptr_t)dtype,
        (uintptr_t)sh.ey,         (uintptr_t)sh.ex,
        (uintptr_t)n,             (uintptr_t)bc,            (uintptr_t)sc.order,       (uintptr_t)frames,
        (uintptr_t)fps,           (uintptr_t)cand,          (uintptr_t)rec,            (uintptr_t)ws_inter.ptr,
        (uintptr_t)ws_band.ptr,   (uintptr_t)ws_win.ptr,    (uintptr_t)ws_norm.ptr,    (uintptr_t)ws_energy.ptr,
        (uintptr_t)twM,           (uintptr_t)twMi,          (uintptr_t)twN,            (uintptr_t)proj};
    for (GraphEntry& g : graphs)
      if (g.key == key) {
        g.last_use = ++graph_clock;
        if ((e = hipGraphLaunch(g.exec, stream)) != hipSuccess) return ctx.hip_fail(e, "graph launch");
        ++graph_replays;
        return PRNU_OK;
      }
    // Capture only a launch set seen before: one that does not repeat runs eagerly.
    auto seen_it = std::find(seen.begin(), seen.end(), key);
    if (seen_it == seen.end()) {
      if (seen.size() >= kMaxSeen) seen.erase(seen.begin());
      seen.push_back(key);
      if ((e = launch_all(sh, dtype, frames, fps, cand, proj, rec, n, sc, twM, twMi, twN)) != hipSuccess)
        return ctx.hip_fail(e, "search launch");
      return PRNU_OK;
    }
    seen.erase(seen_it);
    if ((e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return ctx.hip_fail(e, "graph capture");
    const hipError_t le = launch_all(sh, dtype, frames, fps, cand, proj, rec, n, sc, twM, twMi, twN);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(stream, &graph);
    if (le != hipSuccess || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return ctx.hip_fail(le != hipSuccess ? le : e, "graph capture");
    }
    GraphEntry ge;
    ge.key = key;
    e = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return ctx.hip_fail(e, "graph instantiate");
    if (graphs.size() >= kMaxGraphs) {
      // evict the least recently used (after the stream has finished any launch of it)
      auto lru = std::min_element(graphs.begin(), graphs.end(),
                                  [](const GraphEntry& x, const GraphEntry& y) { return x.last_use < y.last_use; });
      (void)hipStreamSynchronize(stream);
      (void)hipGraphExecDestroy(lru->exec);
      graphs.erase(lru);
    }
    ge.last_use = ++graph_clock;
    graphs.push_back(ge);
    ++graph_captures;
    if ((e = hipGraphLaunch(ge.exec, stream)) != hipSuccess) return ctx.hip_fail(e, "graph launch");
    return PRNU_OK;
  }
  // Profiled: eager launches bracketed by events per kernel.
  const double MN = (double)sh.M * sh.N, MH = (double)sh.M * sh.Nh() * 8.0;
  const double band = (double)sh.band_rows() * sh.Nh() * 8.0;
  const double res = MN * (dtype == PRNU_BF16 ? 2.0 : 4.0);
  const double win = (double)sh.band_rows() * sh.win_cols() * 4.0;
  for (int start = 0; start < n; start += bc) {
    const int nc = std::min(bc, n - start);
    const Batch b = make_batch(*this, sh, dtype, frames, fps, cand, proj, rec, start, nc, sc.order, twM, twMi, twN);
    prof_begin(0);
    if ((e = launch_warp_rowfft(b, stream)) != hipSuccess) return ctx.hip_fail(e, "warp+row FFT launch");
    prof_end(0, nc, nc * (res + MH));
    prof_begin(1);
    if ((e = launch_col_product(b, stream)) != hipSuccess) return ctx.hip_fail(e, "column FFT launch");
    prof_end(1, nc, nc * (2.0 * MH + band));
    prof_begin(2);
    if ((e = launch_band_rowifft(b, stream)) != hipSuccess) return ctx.hip_fail(e, "band row FFT launch");
    prof_end(2, nc, nc * (band + win));
    prof_begin(3);
    if ((e = launch_pce(b, stream)) != hipSuccess) return ctx.hip_fail(e, "PCE launch");
    prof_end(3, nc, nc * win);
  }
  return PRNU_OK;
}

prnu_status Runner::run_dyn(Context& ctx, const Shape& sh, int dtype, const FrameRef* frames, const FpRef* fps,
                            const CandParam* cand, CandRecord* rec, int n_max, const int* n_dev, int n_full) {
  if (n_max <= 0) return PRNU_OK;
  Schedule sc;
  prnu_status st = ctx.schedule(sh, dtype, *this, sc);
  if (st != PRNU_OK) return st;
  if (batch_override > 0) sc.chunk = batch_override;
  if ((st = ensure_workspace(sh, std::min(sc.chunk, n_max))) != PRNU_OK) return st;
  const c32* twM = ctx.twiddles(kColPlan, sh.M);
  const c32* twMi = ctx.twiddles(kColPlanRev, sh.M);
  const c32* twN = ctx.twiddles(kRowPlan, sh.N);
  if (!twM || !twMi || !twN) return ctx.hip_fail(hipErrorOutOfMemory, "twiddle tables");
  for (int start = 0; start < n_max; start += sc.chunk) {
    const int nc = std::min(sc.chunk, n_max - start);
    Batch b = make_batch(*this, sh, dtype, frames, fps, cand, nullptr, rec, start, nc, sc.order, twM, twMi, twN);
    b.nc_dev = n_dev;
    b.dyn_start = start;
    b.dyn_full = start < n_full ? 1 : 0;
    hipError_t e;
    if ((e = launch_warp_rowfft(b, stream)) != hipSuccess || (e = launch_col_product(b, stream)) != hipSuccess ||
        (e = launch_band_rowifft(b, stream)) != hipSuccess || (e = launch_pce(b, stream)) != hipSuccess)
      return ctx.hip_fail(e, "fallback launch");
  }
  return PRNU_OK;
}

prnu_status Runner::step(Context& ctx, const Shape& sh, int dtype, const FrameRef* frames, const FpRef* fps,
                         const StepDev& d) {
  hipError_t e;
  if ((e = launch_gen(d.items, d.n_items, d.max_n, d.cand, d.site, stream)) != hipSuccess)
    return ctx.hip_fail(e, "candidate generation");
  prnu_status st = run(ctx, sh, dtype, frames, fps, d.cand, d.rec, d.n_total);
  if (st != PRNU_OK) return st;
  if ((e = launch_argmax(d.items, d.n_items, d.outs, d.rec, d.site, false, nullptr, nullptr, stream)) != hipSuccess)
    return ctx.hip_fail(e, "argmax");
  if (d.max_fb <= 0) return PRNU_OK;
  if ((e = launch_plan(d.items, d.n_items, d.outs, d.n_dev, stream)) != hipSuccess ||
      (e = launch_fill(d.items, d.n_items, d.outs, d.n_dev, d.max_fb, d.fb_cand, d.fb_site, stream)) != hipSuccess)
    return ctx.hip_fail(e, "fallback plan");
  if ((st = run_dyn(ctx, sh, dtype, frames, fps, d.fb_cand, d.fb_rec, d.max_fb, d.n_dev, d.fb_expect)) != PRNU_OK)
    return st;
  if ((e = launch_argmax(d.items, d.n_items, d.outs, nullptr, nullptr, true, d.fb_rec, d.fb_site, stream)) !=
      hipSuccess)
    return ctx.hip_fail(e, "argmax");
  return PRNU_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: schedules per shape, timed on synthetic data, cached in a text file.

prnu_status Context::schedule(const Shape& sh, int dtype, Runner& r, Schedule& out) {
  if (sh.padded()) {
    // Smaller frames run the same kernels on the same transform size with a larger
    // band and window: the equal-size schedule, its batch capped so that the larger
    // workspace still fits the tuning limit.
    Shape base{sh.M, sh.N, sh.radius};
    prnu_status st = schedule(base, dtype, r, out);
    if (st != PRNU_OK) return st;
    while (out.chunk > 1 && r.workspace_bytes(sh, out.chunk) > tune_cap_bytes) out.chunk = (out.chunk + 1) / 2;
    return PRNU_OK;
  }
  const ShapeKey k{sh.M, sh.N, sh.radius, dtype};
  std::lock_guard<std::mutex> lk(tune_mu);
  auto it = schedules.find(k);
  if (it != schedules.end()) {
    // a schedule read from a cache file is held to the same workspace limit as a tuned
    // one (results do not depend on the batch)
    while (it->second.chunk > 1 && r.workspace_bytes(sh, it->second.chunk) > tune_cap_bytes)
      it->second.chunk = (it->second.chunk + 1) / 2;
    out = it->second;
    return PRNU_OK;
  }
  if (flags & PRNU_FLAG_NO_AUTOTUNE) {
    out = Schedule{};
    out.chunk = r.batch_size(sh);
    schedules[k] = out;
    return PRNU_OK;
  }
  prnu_status st = tune(sh, dtype, r, out);
  if (st != PRNU_OK) return st;
  schedules[k] = out;
  save_tune_cache();
  return PRNU_OK;
}

// Times every schedule whose workspace fits tune_cap_bytes: FFT batches of 8..768
// candidates, both block orders.  The data are zeros (a zero frame, a zero fingerprint
// spectrum): the kernels have no value-dependent control flow, so their time is that
// of real data, while the candidate list spans the full grid's scales and rotations so
// that the warp's access pattern is the real one.  Called with tune_mu held.
prnu_status Context::tune(const Shape& sh, int dtype, Runner& r, Schedule& out) {
  static const int kChunks[] = {8, 16, 32, 48, 64, 96, 128, 192, 256, 320, 384, 448, 512, 640, 768};
  int maxc = 0;
  for (int c : kChunks)
    if (r.workspace_bytes(sh, c) <= tune_cap_bytes) maxc = c;
  if (maxc == 0) maxc = 1;
  const size_t esz = dtype == PRNU_BF16 ? 2 : 4;
  struct Tables {
    FrameRef f;
    FpRef p;
    float one;
  };
  DevBuf frame, fk, tables, cand, rec;
  hipError_t e;
  hipStream_t s = r.stream;
  if ((e = frame.reserve((size_t)padded_frame(sh.M, sh.N) * esz)) != hipSuccess ||
      (e = fk.reserve((size_t)sh.M * tiled_cols(sh) * sizeof(c32))) != hipSuccess ||
      (e = tables.reserve(sizeof(Tables))) != hipSuccess ||
      (e = cand.reserve(sizeof(CandParam) * (size_t)maxc)) != hipSuccess ||
      (e = rec.reserve(sizeof(CandRecord) * (size_t)maxc)) != hipSuccess)
    return fail(PRNU_E_NOMEM, "tuning buffers: %s", hipGetErrorString(e));
  Tables* dt = reinterpret_cast<Tables*>(tables.ptr);
  const Tables ht = {FrameRef{frame.ptr, dtype == PRNU_BF16 ? &dt->one : nullptr},
                     FpRef{reinterpret_cast<c32*>(fk.ptr), 1.0}, 1.0f};
  std::vector<CandParam> hc((size_t)maxc);
  for (int i = 0; i < maxc; ++i) {
    const int a = (i * 7) % 41, t = (i * 3) % 21;  // spread over the 41 x 21 grid
    hc[(size_t)i] = make_param(Cand{grid_node(a, 41, 0.85, 1.15), grid_node(t, 21, -2.0, 2.0)}, 0, 0);
  }
  if ((e = hipMemsetAsync(frame.ptr, 0, frame.cap, s)) != hipSuccess ||
      (e = hipMemsetAsync(fk.ptr, 0, fk.cap, s)) != hipSuccess ||
      (e = hipMemcpyAsync(tables.ptr, &ht, sizeof(ht), hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(cand.ptr, hc.data(), sizeof(CandParam) * (size_t)maxc, hipMemcpyHostToDevice, s)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "tuning setup");
  const c32* twM = twiddles(kColPlan, sh.M);
  const c32* twMi = twiddles(kColPlanRev, sh.M);
  const c32* twN = twiddles(kRowPlan, sh.N);
  if (!twM || !twMi || !twN) return hip_fail(hipErrorOutOfMemory, "twiddle tables");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(e, "tuning events");
  }
  const FrameRef* dframes = &dt->f;
  const FpRef* dfps = &dt->p;
  const CandParam* dcand = reinterpret_cast<const CandParam*>(cand.ptr);
  CandRecord* drec = reinterpret_cast<CandRecord*>(rec.ptr);
  std::vector<Schedule> timed;
  prnu_status st = PRNU_OK;
  for (int c : kChunks) {
    if (c > maxc) break;
    if ((st = r.ensure_workspace(sh, c)) != PRNU_OK) break;
    // each timing covers at least 2 maxc candidates (tens of milliseconds at 1080p)
    const int reps = std::max(4, (2 * maxc + c - 1) / c);
    for (int order = 0; order < 2 && st == PRNU_OK; ++order) {
      Schedule sc;
      sc.chunk = c;
      sc.order = order;
      float ms = 0.f;
      if ((e = r.launch_all(sh, dtype, dframes, dfps, dcand, nullptr, drec, c, sc, twM, twMi, twN)) != hipSuccess ||
          (e = hipEventRecord(e0, s)) != hipSuccess) {
        st = hip_fail(e, "tuning launch");
        break;
      }
      for (int k = 0; k < reps && e == hipSuccess; ++k) e = r.launch_all(sh, dtype, dframes, dfps, dcand, nullptr, drec, c, sc, twM, twMi, twN);
      if (e != hipSuccess || (e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
          (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
        st = hip_fail(e, "tuning launch");
        break;
      }
      sc.ns_per_cand = (double)ms * 1e6 / ((double)reps * c);
      timed.push_back(sc);
    }
    if (st != PRNU_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != PRNU_OK) return st;
  if (timed.empty()) return fail(PRNU_E_NOMEM, "no schedule fits the tuning memory cap");
  // Schedules within 2% of the fastest are ties (timing noise, and the spread between
  // runs on one box): take the largest batch among them (fewest launches), then block
  // order 0, so the choice is reproducible.
  double fastest = timed[0].ns_per_cand;
  for (const Schedule& t : timed) fastest = std::min(fastest, t.ns_per_cand);
  Schedule best = timed[0];
  bool have = false;
  for (const Schedule& t : timed) {
    if (t.ns_per_cand > fastest * 1.02) continue;
    if (!have || t.chunk > best.chunk || (t.chunk == best.chunk && t.order < best.order)) best = t;
    have = true;
  }
  out = best;
  return PRNU_OK;
}

// Cache file: one schedule per line, "M N radius dtype chunk order ns_per_candidate".
void Context::load_tune_cache() {
  if (tune_cache.empty()) return;
  FILE* f = std::fopen(tune_cache.c_str(), "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof(line), f)) {
    if (line[0] == '#') continue;
    int M, N, R, dt, chunk, order;
    double ns;
    if (std::sscanf(line, "%d %d %d %d %d %d %lf", &M, &N, &R, &dt, &chunk, &order, &ns) != 7) continue;
    if (chunk < 1 || chunk > 4096 || (order != 0 && order != 1)) continue;
    Schedule sc;
    sc.chunk = chunk;
    sc.order = order;
    sc.ns_per_cand = ns;
    sc.from_cache = true;
    schedules[ShapeKey{M, N, R, dt}] = sc;
  }
  std::fclose(f);
}

void Context::save_tune_cache() {
  if (tune_cache.empty()) return;
  const std::string tmp = tune_cache + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "# search launch schedules: M N radius dtype batch order ns_per_candidate\n");
  for (auto& kv : schedules) {
    if (kv.second.ns_per_cand <= 0.0) continue;
    std::fprintf(f, "%d %d %d %d %d %d %.1f\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
                 std::get<3>(kv.first), kv.second.chunk, kv.second.order, kv.second.ns_per_cand);
  }
  std::fclose(f);
  (void)std::rename(tmp.c_str(), tune_cache.c_str());
}

hipEvent_t Runner::prof_event() {
  if (ev_used == ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ev_pool.push_back(e);
  }
  return ev_pool[ev_used++];
}

void Runner::prof_begin(int k) {
  if (!prof_on) return;
  hipEvent_t a = prof_event();
  if (!a) return;
  (void)hipEventRecord(a, stream);
  prof_pending.push_back(ProfEvent{k, a, nullptr, 0, 0.0});
}

void Runner::prof_end(int k, int nc, double bytes) {
  if (!prof_on || prof_pending.empty() || prof_pending.back().kernel != k || prof_pending.back().stop) return;
  hipEvent_t b = prof_event();
  if (!b) return;
  (void)hipEventRecord(b, stream);
  prof_pending.back().stop = b;
  prof_pending.back().cands = nc;
  prof_pending.back().bytes = bytes;
}

void Runner::prof_collect() {
  for (auto& p : prof_pending) {
    float ms = 0.f;
    if (p.start && p.stop && hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
      prof[p.kernel].launches += 1;
      prof[p.kernel].total_ms += ms;
      prof[p.kernel].candidates += p.cands;
      prof[p.kernel].algo_bytes += p.bytes;
    }
  }
  prof_pending.clear();
  ev_used = 0;
}

// ---------------------------------------------------------------------------
// Context.

const c32* Context::twiddles(int kind, int L) {
  std::lock_guard<std::mutex> lk(tw_mu);
  const int key = kind * 100000 + L;
  auto it = tw.find(key);
  if (it != tw.end()) return it->second;
  const int n = twiddle_table(kind, L, nullptr, 0);
  if (n <= 0) return nullptr;
  std::vector<c32> h((size_t)n);
  twiddle_table(kind, L, h.data(), n);
  void* d = nullptr;
  if (hipMalloc(&d, (size_t)n * sizeof(c32)) != hipSuccess) return nullptr;
  if (hipMemcpy(d, h.data(), (size_t)n * sizeof(c32), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return nullptr;
  }
  tw[key] = reinterpret_cast<c32*>(d);
  return reinterpret_cast<c32*>(d);
}

const c32* Context::find_twiddles(int kind, int L) {
  std::lock_guard<std::mutex> lk(tw_mu);
  auto it = tw.find(kind * 100000 + L);
  return it == tw.end() ? nullptr : it->second;
}

bool Context::get_fp(prnu_fp h, Fingerprint& out) {
  std::lock_guard<std::mutex> lk(fp_mu);
  auto it = fps.find(h);
  if (it == fps.end()) return false;
  out = it->second;
  return true;
}

// Make stream s wait for the work already queued on the caller's stream.  A null
// caller stream is the legacy default stream (torch's default stream), which the
// library's non-blocking streams do not synchronise with by themselves.
static prnu_status order_after(Context& ctx, hipStream_t s, void* caller) {
  hipEvent_t ev;
  hipError_t e;
  if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return ctx.hip_fail(e, "event create");
  if ((e = hipEventRecord(ev, (hipStream_t)caller)) != hipSuccess || (e = hipStreamWaitEvent(s, ev, 0)) != hipSuccess) {
    (void)hipEventDestroy(ev);
    return ctx.hip_fail(e, "stream ordering");
  }
  (void)hipEventDestroy(ev);
  return PRNU_OK;
}

// F host frames of M x N elements of esz bytes (frame and row strides in elements) into
// the tight device buffer dst: the rows are gathered into pinned memory on the host and
// sent in one DMA (row-by-row copies from pageable memory are slow).  The caller
// synchronises s before `pinned` is reused.
static hipError_t upload_tight(hipStream_t s, const void* host, size_t esz, int F, int M, int N, int64_t fs, int64_t rs,
                               HostBuf& pinned, void* dst) {
  const size_t fbytes = (size_t)M * N * esz;
  if (F == 0) return hipSuccess;
  hipError_t e;
  if ((e = pinned.reserve(fbytes * (size_t)F)) != hipSuccess) return e;
  const char* h = reinterpret_cast<const char*>(host);
  char* p = reinterpret_cast<char*>(pinned.ptr);
  for (int f = 0; f < F; ++f) {
    const char* src = h + (size_t)f * fs * esz;
    if (rs == N) {
      std::memcpy(p + (size_t)f * fbytes, src, fbytes);
    } else {
      for (int y = 0; y < M; ++y)
        std::memcpy(p + (size_t)f * fbytes + (size_t)y * N * esz, src + (size_t)y * rs * esz, (size_t)N * esz);
    }
  }
  return hipMemcpyAsync(dst, pinned.ptr, fbytes * (size_t)F, hipMemcpyHostToDevice, s);
}

// An allocation failure is PRNU_E_NOMEM; anything else is a device failure.
static prnu_status staging_fail(Context& ctx, hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return fail(PRNU_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
  return ctx.hip_fail(e, what);
}

prnu_status stage_padded(Context& ctx, hipStream_t s, const prnu_frames* fr, DevBuf& tight, DevBuf& padded,
                         HostBuf* pinned) {
  if (ctx.inject(ctx.fault_stage, ctx.n_stage)) return ctx.hip_fail(hipErrorInvalidValue, "injected staging fault");
  const size_t esz = fr->dtype == PRNU_BF16 ? 2 : 4;
  const int M = fr->height, N = fr->width, F = fr->n_frames;
  hipError_t e;
  if ((e = padded.reserve((size_t)padded_frame(M, N) * esz * (size_t)std::max(F, 1))) != hipSuccess)
    return fail(PRNU_E_NOMEM, "frame staging: %s", hipGetErrorString(e));
  const void* from = fr->data;
  int64_t fs = fr->frame_stride, rs = fr->row_stride;
  if (fr->on_device) {
    prnu_status st = order_after(ctx, s, fr->stream);
    if (st != PRNU_OK) return st;
  } else {
    const size_t fbytes = (size_t)M * N * esz;
    if ((e = tight.reserve(fbytes * (size_t)std::max(F, 1))) != hipSuccess)
      return fail(PRNU_E_NOMEM, "frame upload: %s", hipGetErrorString(e));
    const char* h = reinterpret_cast<const char*>(fr->data);
    if (pinned) {
      // pageable caller memory (the synchronous calls synchronise before reuse)
      if ((e = upload_tight(s, h, esz, F, M, N, fr->frame_stride, fr->row_stride, *pinned, tight.ptr)) != hipSuccess)
        return staging_fail(ctx, e, "frame upload");
    } else if (fr->row_stride == N && (F == 1 || fr->frame_stride == (int64_t)M * N)) {
      // tight (the serving engine's pinned copy): one DMA
      if (F > 0 && (e = hipMemcpyAsync(tight.ptr, h, fbytes * (size_t)F, hipMemcpyHostToDevice, s)) != hipSuccess)
        return ctx.hip_fail(e, "frame upload");
    } else {
      for (int f = 0; f < F; ++f) {
        e = hipMemcpy2DAsync(reinterpret_cast<char*>(tight.ptr) + (size_t)f * fbytes, (size_t)N * esz,
                             h + (size_t)f * fr->frame_stride * esz, (size_t)fr->row_stride * esz, (size_t)N * esz,
                             (size_t)M, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return ctx.hip_fail(e, "frame upload");
      }
    }
    from = tight.ptr;
    fs = (int64_t)M * N;
    rs = N;
  }
  if ((e = launch_pad_frames(from, (int)esz, fs, rs, F, M, N, padded.ptr, s)) != hipSuccess)
    return ctx.hip_fail(e, "frame staging");
  return PRNU_OK;
}

// Stage a video's frames for the synchronous path; refs[f] describes frame f.
prnu_status Context::stage_frames(const prnu_frames* fr, std::vector<FrameRef>& refs) {
  prnu_status st = stage_padded(*this, runner.stream, fr, stage_tight, stage_dev, &stage_pinned);
  if (st != PRNU_OK) return st;
  const int F = fr->n_frames;
  const size_t fbytes = (size_t)padded_frame(fr->height, fr->width) * (fr->dtype == PRNU_BF16 ? 2 : 4);
  const float* scales = nullptr;
  if (fr->dtype == PRNU_BF16) {
    if (fr->on_device) {
      scales = fr->frame_scale;
    } else {
      hipError_t e;
      if ((e = stage_scale.reserve(sizeof(float) * (size_t)std::max(1, F))) != hipSuccess)
        return fail(PRNU_E_NOMEM, "scale staging");
      if (F > 0 && (e = hipMemcpyAsync(stage_scale.ptr, fr->frame_scale, sizeof(float) * (size_t)F,
                                       hipMemcpyHostToDevice, runner.stream)) != hipSuccess)
        return hip_fail(e, "scale upload");
      scales = reinterpret_cast<const float*>(stage_scale.ptr);
    }
  }
  refs.resize((size_t)F);
  for (int f = 0; f < F; ++f)
    refs[(size_t)f] = FrameRef{reinterpret_cast<const char*>(stage_dev.ptr) + (size_t)f * fbytes,
                               scales ? scales + f : nullptr};
  return PRNU_OK;
}

prnu_status Context::upload_refs(const std::vector<FrameRef>& frames, const Fingerprint& fp) {
  const size_t fb = sizeof(FrameRef) * std::max<size_t>(1, frames.size());
  hipError_t e;
  if ((e = host_refs.reserve(fb + sizeof(FpRef))) != hipSuccess || (e = dev_frefs.reserve(fb)) != hipSuccess ||
      (e = dev_fprefs.reserve(sizeof(FpRef))) != hipSuccess)
    return fail(PRNU_E_NOMEM, "frame tables");
  char* h = reinterpret_cast<char*>(host_refs.ptr);
  if (!frames.empty()) std::memcpy(h, frames.data(), sizeof(FrameRef) * frames.size());
  const FpRef fr{fp.FK, fp.norm};
  std::memcpy(h + fb, &fr, sizeof(fr));
  if ((e = hipMemcpyAsync(dev_frefs.ptr, h, fb, hipMemcpyHostToDevice, runner.stream)) != hipSuccess ||
      (e = hipMemcpyAsync(dev_fprefs.ptr, h + fb, sizeof(FpRef), hipMemcpyHostToDevice, runner.stream)) != hipSuccess)
    return hip_fail(e, "frame tables");
  return PRNU_OK;
}

// Evaluate explicit candidate lists against the uploaded frame / fingerprint tables,
// synchronously.
prnu_status Context::evaluate(const Shape& sh, int dtype, const std::vector<CandParam>& params,
                              std::vector<CandRecord>& recs, const std::vector<float>* proj) {
  const int n = (int)params.size();
  recs.assign((size_t)n, CandRecord{});
  if (n == 0) return PRNU_OK;
  hipError_t e;
  if ((e = host_cand.reserve(sizeof(CandParam) * (size_t)n)) != hipSuccess) return fail(PRNU_E_NOMEM, "pinned");
  if ((e = host_rec.reserve(sizeof(CandRecord) * (size_t)n)) != hipSuccess) return fail(PRNU_E_NOMEM, "pinned");
  if ((e = dev_cand.reserve(sizeof(CandParam) * (size_t)n)) != hipSuccess) return fail(PRNU_E_NOMEM, "candidates");
  if ((e = dev_rec.reserve(sizeof(CandRecord) * (size_t)n)) != hipSuccess) return fail(PRNU_E_NOMEM, "records");
  std::memcpy(host_cand.ptr, params.data(), sizeof(CandParam) * (size_t)n);
  if ((e = hipMemcpyAsync(dev_cand.ptr, host_cand.ptr, sizeof(CandParam) * (size_t)n, hipMemcpyHostToDevice,
                          runner.stream)) != hipSuccess)
    return hip_fail(e, "candidate upload");
  const float* dproj = nullptr;
  if (proj) {
    if ((e = dev_proj.reserve(sizeof(float) * proj->size())) != hipSuccess) return fail(PRNU_E_NOMEM, "transforms");
    if ((e = hipMemcpyAsync(dev_proj.ptr, proj->data(), sizeof(float) * proj->size(), hipMemcpyHostToDevice,
                            runner.stream)) != hipSuccess)
      return hip_fail(e, "transform upload");
    dproj = reinterpret_cast<const float*>(dev_proj.ptr);
  }
  prnu_status st = runner.run(*this, sh, dtype, reinterpret_cast<FrameRef*>(dev_frefs.ptr),
                              reinterpret_cast<FpRef*>(dev_fprefs.ptr), reinterpret_cast<CandParam*>(dev_cand.ptr),
                              reinterpret_cast<CandRecord*>(dev_rec.ptr), n, dproj);
  if (st != PRNU_OK) return st;
  if ((e = hipMemcpyAsync(host_rec.ptr, dev_rec.ptr, sizeof(CandRecord) * (size_t)n, hipMemcpyDeviceToHost,
                          runner.stream)) != hipSuccess)
    return hip_fail(e, "record download");
  if ((e = hipStreamSynchronize(runner.stream)) != hipSuccess) return hip_fail(e, "search");
  runner.prof_collect();
  std::memcpy(recs.data(), host_rec.ptr, sizeof(CandRecord) * (size_t)n);
  return PRNU_OK;
}

// Synchronous-path buffers for n_items items, a candidate list of n_total, a fallback
// list of max_fb, F frames (results and running bests) and list_sites explicit
// candidate sites.
static prnu_status reserve_sync(Context& c, int n_items, int n_total, int max_fb, int F, size_t list_sites) {
  const size_t ni = (size_t)std::max(1, n_items), nt = (size_t)std::max(1, n_total), nb = (size_t)std::max(1, max_fb),
               nf = (size_t)std::max(1, F), nl = std::max<size_t>(1, list_sites);
  hipError_t e;
  if ((e = c.dev_items.reserve(sizeof(ItemDesc) * ni)) != hipSuccess ||
      (e = c.dev_outs.reserve(sizeof(ItemOut) * ni)) != hipSuccess ||
      (e = c.dev_cand.reserve(sizeof(CandParam) * nt)) != hipSuccess ||
      (e = c.dev_site.reserve(sizeof(CandSite) * nt)) != hipSuccess ||
      (e = c.dev_rec.reserve(sizeof(CandRecord) * nt)) != hipSuccess ||
      (e = c.dev_fbc.reserve(sizeof(CandParam) * nb)) != hipSuccess ||
      (e = c.dev_fbs.reserve(sizeof(CandSite) * nb)) != hipSuccess ||
      (e = c.dev_fbr.reserve(sizeof(CandRecord) * nb)) != hipSuccess ||
      (e = c.dev_ndev.reserve(sizeof(int))) != hipSuccess ||
      (e = c.dev_state.reserve(sizeof(ChainState))) != hipSuccess ||
      (e = c.dev_best.reserve(sizeof(FrameBest) * nf)) != hipSuccess ||
      (e = c.dev_res.reserve(sizeof(prnu_frame_result) * nf)) != hipSuccess ||
      (e = c.dev_lists.reserve(sizeof(CandSite) * nl)) != hipSuccess ||
      (e = c.host_items.reserve(sizeof(ItemDesc) * ni)) != hipSuccess ||
      (e = c.host_outs.reserve(sizeof(ItemOut) * ni)) != hipSuccess ||
      (e = c.host_res.reserve(sizeof(prnu_frame_result) * nf)) != hipSuccess ||
      (e = c.host_lists.reserve(sizeof(CandSite) * nl)) != hipSuccess)
    return fail(PRNU_E_NOMEM, "search buffers: %s", hipGetErrorString(e));
  return PRNU_OK;
}

static StepDev sync_step(Context& c) {
  StepDev d;
  d.items = reinterpret_cast<const ItemDesc*>(c.dev_items.ptr);
  d.outs = reinterpret_cast<ItemOut*>(c.dev_outs.ptr);
  d.cand = reinterpret_cast<CandParam*>(c.dev_cand.ptr);
  d.site = reinterpret_cast<CandSite*>(c.dev_site.ptr);
  d.rec = reinterpret_cast<CandRecord*>(c.dev_rec.ptr);
  d.fb_cand = reinterpret_cast<CandParam*>(c.dev_fbc.ptr);
  d.fb_site = reinterpret_cast<CandSite*>(c.dev_fbs.ptr);
  d.fb_rec = reinterpret_cast<CandRecord*>(c.dev_fbr.ptr);
  d.n_dev = reinterpret_cast<int*>(c.dev_ndev.ptr);
  return d;
}

// The results of F frames written on the device, to out (synchronises the stream).
static prnu_status download_results(Context& c, int F, prnu_frame_result* out) {
  hipError_t e;
  if (F > 0 && (e = hipMemcpyAsync(c.host_res.ptr, c.dev_res.ptr, sizeof(prnu_frame_result) * (size_t)F,
                                   hipMemcpyDeviceToHost, c.runner.stream)) != hipSuccess)
    return c.hip_fail(e, "result download");
  if ((e = hipStreamSynchronize(c.runner.stream)) != hipSuccess) return c.hip_fail(e, "search");
  c.runner.prof_collect();
  if (F > 0) std::memcpy(out, c.host_res.ptr, sizeof(prnu_frame_result) * (size_t)F);
  return PRNU_OK;
}

// The coarse-to-fine schedule on F staged frames, frame f starting from inits[f]: each
// iteration's grids of all unfinished frames are searched in one launch; the device
// reduces every frame's grid to its best candidate, folds it into the frame's best over
// all iterations and writes the frame's result; the host moves each frame to its
// iteration's best or stops it.
prnu_status Context::refine(const Shape& sh, int dtype, int F, const prnu_search_opts* o,
                            const std::vector<std::pair<double, double>>& inits, prnu_frame_result* out) {
  if (F == 0) return PRNU_OK;
  struct FrameState {
    double cs, ct;
    bool done = false;
  };
  std::vector<FrameState> fs((size_t)F);
  for (int f = 0; f < F; ++f) {
    fs[(size_t)f].cs = inits[(size_t)f].first;
    fs[(size_t)f].ct = inits[(size_t)f].second;
  }
  std::vector<Cand> grid;
  std::vector<CandSite> sites;
  prnu_status st;
  hipError_t e;
  hipStream_t s = runner.stream;
  for (int n = 1; n <= o->refine_max_iter; ++n) {
    std::vector<int> who;
    std::vector<ItemDesc> items;
    sites.clear();
    for (int f = 0; f < F; ++f) {
      FrameState& x = fs[(size_t)f];
      if (x.done) continue;
      refine_candidates(*o, n, x.cs, x.ct, grid);
      ItemDesc it{};
      it.gen.kind = kGenList;
      it.n = (int)grid.size();
      it.off = (int)sites.size();
      it.slot = f;
      it.fslot = 0;
      it.mode = kModeRefine;
      it.merge = n > 1;
      it.iter = n;
      for (const Cand& c : grid) sites.push_back(CandSite{c.scale, c.rot_deg});
      items.push_back(it);
      who.push_back(f);
    }
    if (who.empty()) break;
    const int ni = (int)items.size(), nt = (int)sites.size();
    int max_n = 0;
    for (const ItemDesc& it : items) max_n = std::max(max_n, it.n);
    if ((st = reserve_sync(*this, ni, nt, 0, F, sites.size())) != PRNU_OK) return st;
    const CandSite* dl = reinterpret_cast<const CandSite*>(dev_lists.ptr);
    FrameBest* best = reinterpret_cast<FrameBest*>(dev_best.ptr);
    prnu_frame_result* res = reinterpret_cast<prnu_frame_result*>(dev_res.ptr);
    for (int i = 0; i < ni; ++i) {
      items[(size_t)i].gen.list = dl + items[(size_t)i].off;
      items[(size_t)i].best = best + who[(size_t)i];
      items[(size_t)i].result = res + who[(size_t)i];
    }
    std::memcpy(host_items.ptr, items.data(), sizeof(ItemDesc) * (size_t)ni);
    std::memcpy(host_lists.ptr, sites.data(), sizeof(CandSite) * (size_t)nt);
    if ((e = hipMemcpyAsync(dev_items.ptr, host_items.ptr, sizeof(ItemDesc) * (size_t)ni, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(dev_lists.ptr, host_lists.ptr, sizeof(CandSite) * (size_t)nt, hipMemcpyHostToDevice, s)) !=
            hipSuccess)
      return hip_fail(e, "refinement upload");
    StepDev d = sync_step(*this);
    d.n_items = ni;
    d.n_total = nt;
    d.max_n = max_n;
    if ((st = runner.step(*this, sh, dtype, reinterpret_cast<FrameRef*>(dev_frefs.ptr),
                          reinterpret_cast<FpRef*>(dev_fprefs.ptr), d)) != PRNU_OK)
      return st;
    if ((e = hipMemcpyAsync(host_outs.ptr, dev_outs.ptr, sizeof(ItemOut) * (size_t)ni, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return hip_fail(e, "refinement");
    runner.prof_collect();
    const ItemOut* ho = reinterpret_cast<const ItemOut*>(host_outs.ptr);
    for (int i = 0; i < ni; ++i) {
      FrameState& x = fs[(size_t)who[(size_t)i]];
      if (ho[i].seg_index < 0) {
        x.done = true;
        continue;
      }
      if (ho[i].seg_s == x.cs && ho[i].seg_t == x.ct) x.done = true;  // the estimate repeats
      x.cs = ho[i].seg_s;
      x.ct = ho[i].seg_t;
    }
  }
  return download_results(*this, F, out);
}

// G = T^-1 of a general Eq. (4) transform (row-major, FP64), rounded once to float;
// false if T is not finite or (numerically) singular.
bool transform_inverse(const double* T, float* G) {
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(T[i])) return false;
  const double a = T[0], b = T[1], c = T[2], d = T[3], e = T[4], f = T[5], g = T[6], h = T[7], k = T[8];
  const double A = e * k - f * h, B = -(d * k - f * g), C = d * h - e * g;
  const double det = a * A + b * B + c * C;
  double scale = 0.0;
  for (int i = 0; i < 9; ++i) scale = std::max(scale, std::fabs(T[i]));
  if (!(std::fabs(det) > 1e-12 * scale * scale * scale)) return false;
  const double inv[9] = {A, -(b * k - c * h), b * f - c * e, B, a * k - c * g, -(a * f - c * d),
                         C, -(a * h - b * g), a * e - b * d};
  for (int i = 0; i < 9; ++i) G[i] = (float)(inv[i] / det);
  return true;
}

// Nearest similarity (scale, rotation in degrees) of the linear part of T, in the
// convention t11 = t22 = s cos(theta), t12 = -t21 = s sin(theta).
std::pair<double, double> similarity_of(const double* T) {
  const double th = std::atan2(T[1] - T[3], T[0] + T[4]);
  return {std::sqrt(std::fabs(T[0] * T[4] - T[1] * T[3])), th * (180.0 / 3.14159265358979323846)};
}

prnu_status Context::search(const Fingerprint& fp, const prnu_frames* fr, const prnu_search_opts* o,
                            prnu_frame_result* out) {
  std::vector<FrameRef> refs;
  prnu_status st = stage_frames(fr, refs);
  if (st != PRNU_OK) return st;
  if ((st = upload_refs(refs, fp)) != PRNU_OK) return st;
  const Shape sh = search_shape(fp, fr, o->shift_radius);
  const int F = fr->n_frames;
  if (o->refine) {
    std::vector<std::pair<double, double>> inits((size_t)F, o->has_init ? std::make_pair(o->init_scale, o->init_rot_deg)
                                                                          : std::make_pair(1.0, 0.0));
    return refine(sh, fr->dtype, F, o, inits, out);
  }
  if (F == 0) return PRNU_OK;
  const bool warm = o->warm != 0;
  const int nf = o->full.n_scale * o->full.n_rot;
  const int nl = warm ? o->local_n_scale * o->local_n_rot : 0;
  // plain: every frame's full grid in one launch; warm: one launch per frame
  const int n_total = warm ? std::max(nf, nl) : F * nf;
  if ((st = reserve_sync(*this, F, n_total, warm ? nf : 0, F, 0)) != PRNU_OK) return st;
  ChainState* state = reinterpret_cast<ChainState*>(dev_state.ptr);
  FrameBest* best = reinterpret_cast<FrameBest*>(dev_best.ptr);
  prnu_frame_result* res = reinterpret_cast<prnu_frame_result*>(dev_res.ptr);
  ItemDesc* hi = reinterpret_cast<ItemDesc*>(host_items.ptr);
  const GridGen full = full_gen(o->full);
  for (int f = 0; f < F; ++f) {
    ItemDesc it{};
    it.slot = f;
    it.fslot = 0;
    it.result = res + f;
    if (warm && (f > 0 || o->has_init)) {
      // local grid around the previous frame's result (or the initial transform), with
      // the full grid as the device-decided fallback
      it.gen = local_gen(*o, state);
      it.n = nl;
      it.full = full;
      it.fb_n = nf;
      it.fallback_pce = o->fallback_pce;
      it.mode = kModeWarm;
      it.best = best;
      it.state = state;
    } else {
      it.gen = full;
      it.n = nf;
      it.off = warm ? 0 : f * nf;
      it.mode = kModePlain;
      it.best = best + (warm ? 0 : f);
      it.state = warm ? state : nullptr;
    }
    hi[f] = it;
  }
  hipError_t e;
  hipStream_t s = runner.stream;
  if ((e = hipMemcpyAsync(dev_items.ptr, host_items.ptr, sizeof(ItemDesc) * (size_t)F, hipMemcpyHostToDevice, s)) !=
      hipSuccess)
    return hip_fail(e, "item upload");
  const FrameRef* frefs = reinterpret_cast<FrameRef*>(dev_frefs.ptr);
  const FpRef* fprefs = reinterpret_cast<FpRef*>(dev_fprefs.ptr);
  StepDev d = sync_step(*this);
  if (!warm) {
    d.n_items = F;
    d.n_total = F * nf;
    d.max_n = nf;
    if ((st = runner.step(*this, sh, fr->dtype, frefs, fprefs, d)) != PRNU_OK) return st;
  } else {
    // Algorithm 1's chain: every frame enqueued at once; each frame's candidates come
    // from the state its predecessor left on the device.
    if ((e = launch_chain_init(state, o->has_init, o->has_init ? o->init_scale : 1.0,
                               o->has_init ? o->init_rot_deg : 0.0, s)) != hipSuccess)
      return hip_fail(e, "chain state");
    for (int f = 0; f < F; ++f) {
      StepDev df = d;
      df.items += f;
      df.outs += f;
      df.n_items = 1;
      df.n_total = df.max_n = hi[f].n;
      df.max_fb = hi[f].mode == kModeWarm ? nf : 0;
      if ((st = runner.step(*this, sh, fr->dtype, frefs, fprefs, df)) != PRNU_OK) return st;
    }
  }
  return download_results(*this, F, out);
}

prnu_status Context::score_full(const Shape& sh, int dtype, const prnu_grid& g, int frame,
                                std::vector<CandRecord>& recs) {
  const int n = g.n_scale * g.n_rot;
  prnu_status st = reserve_sync(*this, 1, n, 0, 1, 0);
  if (st != PRNU_OK) return st;
  if ((st = (host_rec.reserve(sizeof(CandRecord) * (size_t)n) == hipSuccess ? PRNU_OK : PRNU_E_NOMEM)) != PRNU_OK)
    return fail(st, "pinned records");
  ItemDesc it{};
  it.gen = full_gen(g);
  it.n = n;
  it.slot = frame;
  it.mode = kModePlain;
  *reinterpret_cast<ItemDesc*>(host_items.ptr) = it;
  hipError_t e;
  hipStream_t s = runner.stream;
  if ((e = hipMemcpyAsync(dev_items.ptr, host_items.ptr, sizeof(ItemDesc), hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = launch_gen(reinterpret_cast<const ItemDesc*>(dev_items.ptr), 1, n, reinterpret_cast<CandParam*>(dev_cand.ptr),
                      reinterpret_cast<CandSite*>(dev_site.ptr), s)) != hipSuccess)
    return hip_fail(e, "candidate generation");
  if ((st = runner.run(*this, sh, dtype, reinterpret_cast<FrameRef*>(dev_frefs.ptr),
                       reinterpret_cast<FpRef*>(dev_fprefs.ptr), reinterpret_cast<CandParam*>(dev_cand.ptr),
                       reinterpret_cast<CandRecord*>(dev_rec.ptr), n)) != PRNU_OK)
    return st;
  if ((e = hipMemcpyAsync(host_rec.ptr, dev_rec.ptr, sizeof(CandRecord) * (size_t)n, hipMemcpyDeviceToHost, s)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "scores");
  runner.prof_collect();
  recs.assign(reinterpret_cast<const CandRecord*>(host_rec.ptr), reinterpret_cast<const CandRecord*>(host_rec.ptr) + n);
  return PRNU_OK;
}

// ---------------------------------------------------------------------------
// Device scratch of the allocation-free grid scoring (prnu_score_grid_noalloc): a fixed
// array in the code object, so that the call itself allocates nothing.  In host code
// `scratch` only names the symbol; its device address, one per device, comes from
// hipGetSymbolAddress at context creation and is what the kernels receive.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
bool g_scratch_looked_up[kMaxDevices];
}  // namespace

// Once per device, with that device current.
static void lookup_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_looked_up[dev]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_scratch_err[dev] = e;
  g_scratch_ptr[dev] = e == hipSuccess ? p : nullptr;
  g_scratch_looked_up[dev] = true;
}

static void* scratch_of(int dev, hipError_t* err) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices || !g_scratch_looked_up[dev]) {
    *err = hipErrorNotInitialized;
    return nullptr;
  }
  *err = g_scratch_err[dev];
  return g_scratch_ptr[dev];
}

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr int kNoAllocMaxCandidates = 65536;

Context::~Context() {
  shutdown_serving();
  for (auto& kv : tw) (void)hipFree(kv.second);
  for (auto& kv : fps) (void)hipFree(kv.second.FK);
  if (runner.stream) (void)hipStreamDestroy(runner.stream);
}

}  // namespace prnu

// ===========================================================================
// C ABI.

using namespace prnu;

extern "C" {

const char* prnu_status_string(prnu_status s) {
  switch (s) {
    case PRNU_OK: return "ok";
    case PRNU_PENDING: return "pending";
    case PRNU_E_ARG: return "invalid argument";
    case PRNU_E_SHAPE: return "unsupported or mismatched shape";
    case PRNU_E_NOMEM: return "out of memory or over budget";
    case PRNU_E_DEVICE: return "device error";
    case PRNU_E_HANDLE: return "unknown handle";
    case PRNU_E_BUSY: return "busy";
    case PRNU_E_NONFINITE: return "non-finite value";
    case PRNU_E_CANCELLED: return "cancelled";
  }
  return "unknown status";
}

const char* prnu_last_error(void) { return g_last_error.c_str(); }

int32_t prnu_supported_lengths(int32_t* out, int32_t cap) { return supported_lengths(out, cap); }

prnu_status prnu_create(const prnu_config* cfg, prnu_ctx** out) {
  if (!out) return fail(PRNU_E_ARG, "null output");
  *out = nullptr;
  const int dev = cfg ? cfg->device : 0;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= 0) return fail(PRNU_E_DEVICE, "no HIP device available (%s)", hipGetErrorString(e));
  if (dev < 0 || dev >= count) return fail(PRNU_E_ARG, "device %d out of range (%d devices)", dev, count);
  if ((e = hipSetDevice(dev)) != hipSuccess) return fail(PRNU_E_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
  Context* c = new Context();
  c->device = dev;
  if (cfg) {
    c->hbm_budget = cfg->hbm_budget_bytes;
    c->max_slots = cfg->max_slots;
    if (cfg->tune_cache_path) c->tune_cache = cfg->tune_cache_path;
    c->flags = cfg->flags;
  }
  c->runner.use_graphs = !(c->flags & PRNU_FLAG_NO_GRAPHS);
  c->load_tune_cache();
  if (c->hbm_budget == 0) c->hbm_budget = 16ull << 30;
  if (c->max_slots <= 0) c->max_slots = 16;
  if (const char* b = std::getenv("PRNU_BATCH")) c->runner.batch_override = std::atoi(b);
  if (const char* f = std::getenv("PRNU_FAULT")) {
    // comma-separated "launch:N" and "stage:N"
    std::string spec(f);
    for (size_t pos = 0; pos < spec.size();) {
      size_t end = spec.find(',', pos);
      if (end == std::string::npos) end = spec.size();
      const std::string item = spec.substr(pos, end - pos);
      const size_t colon = item.find(':');
      if (colon != std::string::npos) {
        const long long n = std::atoll(item.c_str() + colon + 1);
        if (item.compare(0, colon, "launch") == 0) c->fault_launch = n;
        if (item.compare(0, colon, "stage") == 0) c->fault_stage = n;
      }
      pos = end + 1;
    }
  }
  if ((e = hipStreamCreateWithFlags(&c->runner.stream, hipStreamNonBlocking)) != hipSuccess) {
    delete c;
    return fail(PRNU_E_DEVICE, "stream create: %s", hipGetErrorString(e));
  }
  lookup_scratch(dev);
  *out = reinterpret_cast<prnu_ctx*>(c);
  return PRNU_OK;
}

void prnu_destroy(prnu_ctx* ctx) {
  if (!ctx) return;
  Context* c = reinterpret_cast<Context*>(ctx);
  (void)hipSetDevice(c->device);
  c->shutdown_serving();
  if (c->runner.stream) (void)hipStreamSynchronize(c->runner.stream);
  delete c;
}

prnu_status prnu_open_fingerprint(prnu_ctx* ctx, const float* K, int32_t height, int32_t width, int64_t row_stride,
                                  int32_t on_device, void* stream, prnu_fp* out) {
  if (!ctx || !K || !out) return fail(PRNU_E_ARG, "null argument");
  Context* c = reinterpret_cast<Context*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->failed) return fail(PRNU_E_DEVICE, "context failed earlier");
  prnu_status st = check_shape(height, width, 0);
  if (st != PRNU_OK) return st;
  if (row_stride < width) return fail(PRNU_E_ARG, "row stride %lld < width %d", (long long)row_stride, width);
  (void)hipSetDevice(c->device);
  hipStream_t s = c->runner.stream;
  const Shape sh{height, width, 0};
  hipError_t e;
  const c32* twM = c->twiddles(kColPlan, height);
  const c32* twMi = c->twiddles(kColPlanRev, height);
  const c32* twN = c->twiddles(kRowPlan, width);
  if (!twM || !twMi || !twN) return c->hip_fail(hipErrorOutOfMemory, "twiddle tables");
  DevBuf kdev, work, inter, sums, stats, small;
  const float* Kd = K;
  int64_t rs = row_stride;
  if (on_device) {
    // order after the caller's stream (null: the legacy default stream)
    if ((st = order_after(*c, s, stream)) != PRNU_OK) return st;
  } else {
    if ((e = kdev.reserve((size_t)height * width * sizeof(float))) != hipSuccess)
      return fail(PRNU_E_NOMEM, "fingerprint upload");
    if ((e = hipMemcpy2DAsync(kdev.ptr, (size_t)width * 4, K, (size_t)row_stride * 4, (size_t)width * 4,
                              (size_t)height, hipMemcpyHostToDevice, s)) != hipSuccess)
      return c->hip_fail(e, "fingerprint upload");
    Kd = reinterpret_cast<const float*>(kdev.ptr);
    rs = width;
  }
  void* FK = nullptr;
  if ((e = work.reserve((size_t)padded_frame(height, width) * sizeof(float))) != hipSuccess ||
      (e = inter.reserve((size_t)height * tiled_cols(sh) * sizeof(c32))) != hipSuccess ||
      (e = sums.reserve((size_t)(height + 2) * sizeof(double))) != hipSuccess ||
      (e = stats.reserve(2 * sizeof(double))) != hipSuccess ||
      (e = small.reserve(sizeof(CandParam) + sizeof(FrameRef))) != hipSuccess ||
      (e = hipMalloc(&FK, (size_t)height * tiled_cols(sh) * sizeof(c32))) != hipSuccess)
    return fail(PRNU_E_NOMEM, "fingerprint buffers: %s", hipGetErrorString(e));
  struct {
    CandParam id;
    FrameRef wref;
  } hsmall = {CandParam{1.f, 0.f, 0, 0}, FrameRef{work.ptr, nullptr}};
  double hstats[2] = {0, 0};
  const CandParam* did = reinterpret_cast<const CandParam*>(small.ptr);
  const FrameRef* dref = reinterpret_cast<const FrameRef*>(reinterpret_cast<char*>(small.ptr) + sizeof(CandParam));
  if ((e = hipMemcpyAsync(small.ptr, &hsmall, sizeof(hsmall), hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = launch_fp_prepare(Kd, rs, sh, reinterpret_cast<float*>(work.ptr), reinterpret_cast<c32*>(inter.ptr),
                             reinterpret_cast<double*>(sums.ptr), reinterpret_cast<double*>(stats.ptr),
                             reinterpret_cast<c32*>(FK), twM, twMi, twN, did, dref, s)) != hipSuccess ||
      (e = hipMemcpyAsync(hstats, stats.ptr, sizeof(hstats), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess) {
    (void)hipFree(FK);
    return c->hip_fail(e, "fingerprint preparation");
  }
  if (!std::isfinite(hstats[0]) || !std::isfinite(hstats[1])) {
    (void)hipFree(FK);
    return fail(PRNU_E_NONFINITE, "fingerprint holds NaN or Inf");
  }
  Fingerprint f;
  f.M = height;
  f.N = width;
  f.FK = reinterpret_cast<c32*>(FK);
  f.mean = hstats[0];
  f.norm = hstats[1];
  std::lock_guard<std::mutex> lf(c->fp_mu);
  const prnu_fp h = ++c->next_fp;
  c->fps[h] = f;
  *out = h;
  return PRNU_OK;
}

prnu_status prnu_close_fingerprint(prnu_ctx* ctx, prnu_fp fp) {
  if (!ctx) return fail(PRNU_E_ARG, "null context");
  Context* c = reinterpret_cast<Context*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  std::lock_guard<std::mutex> lf(c->fp_mu);
  auto it = c->fps.find(fp);
  if (it == c->fps.end()) return fail(PRNU_E_HANDLE, "unknown fingerprint %llu", (unsigned long long)fp);
  if (it->second.users > 0) return fail(PRNU_E_BUSY, "fingerprint has videos in flight");
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->runner.stream);
  (void)hipFree(it->second.FK);
  c->fps.erase(it);
  return PRNU_OK;
}

prnu_status prnu_search_frames(prnu_ctx* ctx, prnu_fp fp, const prnu_frames* frames, const prnu_search_opts* opts,
                               prnu_frame_result* out, prnu_video_summary* summary) {
  if (!ctx || !frames || !opts || (!out && frames->n_frames > 0)) return fail(PRNU_E_ARG, "null argument");
  Context* c = reinterpret_cast<Context*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->failed) return fail(PRNU_E_DEVICE, "context failed earlier");
  Fingerprint f;
  if (!c->get_fp(fp, f)) return fail(PRNU_E_HANDLE, "unknown fingerprint %llu", (unsigned long long)fp);
  prnu_status st = validate_opts(opts);
  if (st != PRNU_OK) return st;
  if ((st = validate_frames(frames, f, opts->shift_radius)) != PRNU_OK) return st;
  (void)hipSetDevice(c->device);
  if ((st = c->search(f, frames, opts, out)) != PRNU_OK) return st;
  if (summary) {
    double sum = 0.0;
    for (int i = 0; i < frames->n_frames; ++i) sum += out[i].pce;
    summary->n_frames = frames->n_frames;
    summary->mean_pce = frames->n_frames ? sum / frames->n_frames : 0.0;
    summary->decision = summary->mean_pce > opts->tau;
    summary->queue_s = 0.0;
    summary->latency_s = 0.0;
  }
  return PRNU_OK;
}

prnu_status prnu_score_grid(prnu_ctx* ctx, prnu_fp fp, const prnu_frames* frames, int32_t frame,
                            const prnu_search_opts* opts, double* pce, double* rho, int32_t* dx, int32_t* dy) {
  if (!ctx || !frames || !opts || !pce) return fail(PRNU_E_ARG, "null argument");
  Context* c = reinterpret_cast<Context*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->failed) return fail(PRNU_E_DEVICE, "context failed earlier");
  Fingerprint f;
  if (!c->get_fp(fp, f)) return fail(PRNU_E_HANDLE, "unknown fingerprint %llu", (unsigned long long)fp);
  prnu_status st = validate_opts(opts);
  if (st != PRNU_OK) return st;
  if ((st = validate_frames(frames, f, opts->shift_radius)) != PRNU_OK) return st;
  if (frame < 0 || frame >= frames->n_frames) return fail(PRNU_E_ARG, "frame %d out of range", frame);
  (void)hipSetDevice(c->device);
  std::vector<FrameRef> refs;
  if ((st = c->stage_frames(frames, refs)) != PRNU_OK) return st;
  if ((st = c->upload_refs(refs, f)) != PRNU_OK) return st;
  std::vector<CandRecord> recs;
  if ((st = c->score_full(search_shape(f, frames, opts->shift_radius), frames->dtype, opts->full, frame, recs)) !=
      PRNU_OK)
    return st;
  for (size_t i = 0; i < recs.size(); ++i) {
    pce[i] = recs[i].pce;
    if (rho) rho[i] = recs[i].rho;
    if (dx) dx[i] = recs[i].dx;
    if (dy) dy[i] = recs[i].dy;
  }
  return PRNU_OK;
}

prnu_status prnu_score_grid_noalloc(prnu_ctx* ctx, prnu_fp fp, const prnu_frames* frames, int32_t frame,
                                    const prnu_search_opts* opts, double* pce, double* rho, int32_t* dx, int32_t* dy) {
  if (!ctx || !frames || !opts || !pce) return fail(PRNU_E_ARG, "null argument");
  Context* c = reinterpret_cast<Context*>(ctx);
  if (c->failed) return fail(PRNU_E_DEVICE, "context failed earlier");
  Fingerprint f;
  if (!c->get_fp(fp, f)) return fail(PRNU_E_HANDLE, "unknown fingerprint %llu", (unsigned long long)fp);
  prnu_status st = validate_opts(opts);
  if (st != PRNU_OK) return st;
  if ((st = validate_frames(frames, f, opts->shift_radius)) != PRNU_OK) return st;
  if (!frames->on_device) return fail(PRNU_E_ARG, "the allocation-free call takes frames in device memory");
  if (frame < 0 || frame >= frames->n_frames) return fail(PRNU_E_ARG, "frame %d out of range", frame);
  const int n = opts->full.n_scale * opts->full.n_rot;
  if (n > kNoAllocMaxCandidates) return fail(PRNU_E_ARG, "%d candidates exceed the limit of %d", n, kNoAllocMaxCandidates);
  (void)hipSetDevice(c->device);
  hipError_t e;
  unsigned char* base = reinterpret_cast<unsigned char*>(scratch_of(c->device, &e));
  if (!base) return fail(PRNU_E_DEVICE, "scratch address of device %d: %s", c->device, hipGetErrorString(e));
  const Shape sh = search_shape(f, frames, opts->shift_radius);
  const c32* twM = c->find_twiddles(kColPlan, sh.M);
  const c32* twMi = c->find_twiddles(kColPlanRev, sh.M);
  const c32* twN = c->find_twiddles(kRowPlan, sh.N);
  if (!twM || !twMi || !twN) return fail(PRNU_E_SHAPE, "no transform tables for %dx%d", sh.M, sh.N);
  // scratch layout: tables and the item, the zero-bordered frame, the candidate list
  // with its sites and records, then the workspace of one batch of candidates
  const size_t esz = frames->dtype == PRNU_BF16 ? 2 : 4;
  const size_t o_frame = 1024;
  const size_t o_cand = o_frame + round256((size_t)padded_frame(sh.Mf(), sh.Nf()) * esz);
  const size_t o_site = o_cand + round256(sizeof(CandParam) * (size_t)n);
  const size_t o_rec = o_site + round256(sizeof(CandSite) * (size_t)n);
  const size_t o_ws = o_rec + round256(sizeof(CandRecord) * (size_t)n);
  const size_t b_inter = (size_t)sh.M * tiled_cols(sh) * sizeof(c32), b_band = (size_t)sh.band_rows() * sh.Nh() * sizeof(c32),
               b_win = (size_t)sh.band_rows() * sh.win_cols() * sizeof(float),
               b_norm = (size_t)sh.row_pairs() * sizeof(double2), b_energy = (size_t)col_blocks(sh) * sizeof(double);
  const size_t per = b_inter + b_band + b_win + b_norm + b_energy;
  const size_t slack = 5 * 256;
  if (o_ws + slack + per > kScratchBytes)
    return fail(PRNU_E_NOMEM, "frame %dx%d against %dx%d needs more than the %zu-byte scratch", frames->height,
                frames->width, sh.M, sh.N, kScratchBytes);
  const int chunk = (int)std::min<size_t>((size_t)n, (kScratchBytes - o_ws - slack) / per);
  unsigned char* ws = base + o_ws;
  c32* inter = reinterpret_cast<c32*>(ws);
  c32* band = reinterpret_cast<c32*>(ws + round256(b_inter * chunk));
  float* win = reinterpret_cast<float*>(reinterpret_cast<unsigned char*>(band) + round256(b_band * chunk));
  double2* norm = reinterpret_cast<double2*>(reinterpret_cast<unsigned char*>(win) + round256(b_win * chunk));
  double* energy = reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(norm) + round256(b_norm * chunk));
  hipStream_t s = reinterpret_cast<hipStream_t>(frames->stream);
  // frame table, fingerprint table and the grid's item, written by a kernel from its
  // arguments
  struct Header {
    FrameRef fr;
    FpRef fpr;
    unsigned char pad[32];
    ItemDesc item;
  } h{};
  const char* src = reinterpret_cast<const char*>(frames->data) + (size_t)frame * frames->frame_stride * esz;
  h.fr = FrameRef{base + o_frame, frames->dtype == PRNU_BF16 ? frames->frame_scale + frame : nullptr};
  h.fpr = FpRef{f.FK, f.norm};
  h.item.gen = full_gen(opts->full);
  h.item.n = n;
  h.item.mode = kModePlain;
  static_assert(sizeof(Header) <= (size_t)kBlobBytes && sizeof(Header) <= 1024, "header");
  Blob blob;
  std::memcpy(blob.b, &h, sizeof(h));
  blob.n = (int32_t)sizeof(h);
  const FrameRef* dframes = reinterpret_cast<const FrameRef*>(base);
  const FpRef* dfps = reinterpret_cast<const FpRef*>(base + offsetof(Header, fpr));
  const ItemDesc* ditem = reinterpret_cast<const ItemDesc*>(base + offsetof(Header, item));
  CandParam* cand = reinterpret_cast<CandParam*>(base + o_cand);
  CandRecord* rec = reinterpret_cast<CandRecord*>(base + o_rec);
  if ((e = launch_put(blob, base, s)) != hipSuccess ||
      (e = launch_pad_frames(src, (int)esz, frames->frame_stride, frames->row_stride, 1, sh.Mf(), sh.Nf(),
                             base + o_frame, s)) != hipSuccess ||
      (e = launch_gen(ditem, 1, n, cand, reinterpret_cast<CandSite*>(base + o_site), s)) != hipSuccess)
    return c->hip_fail(e, "allocation-free scoring");
  for (int start = 0; start < n; start += chunk) {
    Batch b{};
    b.shape = sh;
    b.nc = std::min(chunk, n - start);
    b.cand = cand + start;
    b.dtype = frames->dtype;
    b.frames = dframes;
    b.fps = dfps;
    b.inter = inter;
    b.band = band;
    b.win = win;
    b.norm_part = norm;
    b.energy_part = energy;
    b.rec = rec + start;
    b.twM = twM;
    b.twMi = twMi;
    b.twN = twN;
    if ((e = launch_warp_rowfft(b, s)) != hipSuccess || (e = launch_col_product(b, s)) != hipSuccess ||
        (e = launch_band_rowifft(b, s)) != hipSuccess || (e = launch_pce(b, s)) != hipSuccess)
      return c->hip_fail(e, "allocation-free scoring");
  }
  if ((e = launch_scatter(rec, n, pce, rho, dx, dy, s)) != hipSuccess) return c->hip_fail(e, "allocation-free scoring");
  return PRNU_OK;
}

prnu_status prnu_score_transforms(prnu_ctx* ctx, prnu_fp fp, const prnu_frames* frames, int32_t frame,
                                  const double* T, int32_t n, int32_t shift_radius, double* pce, double* rho,
                                  int32_t* dx, int32_t* dy) {
  if (!ctx || !frames || (n > 0 && (!T || !pce))) return fail(PRNU_E_ARG, "null argument");
  if (n < 0 || n > (1 << 20)) return fail(PRNU_E_ARG, "transform count %d out of range", n);
  Context* c = reinterpret_cast<Context*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->failed) return fail(PRNU_E_DEVICE, "context failed earlier");
  Fingerprint f;
  if (!c->get_fp(fp, f)) return fail(PRNU_E_HANDLE, "unknown fingerprint %llu", (unsigned long long)fp);
  prnu_status st = validate_frames(frames, f, shift_radius);
  if (st != PRNU_OK) return st;
  if (frame < 0 || frame >= frames->n_frames) return fail(PRNU_E_ARG, "frame %d out of range", frame);
  std::vector<float> proj((size_t)n * 9);
  for (int i = 0; i < n; ++i)
    if (!transform_inverse(T + (size_t)i * 9, proj.data() + (size_t)i * 9))
      return fail(PRNU_E_ARG, "transform %d is not finite or not invertible", i);
  if (n == 0) return PRNU_OK;
  (void)hipSetDevice(c->device);
  std::vector<FrameRef> refs;
  if ((st = c->stage_frames(frames, refs)) != PRNU_OK) return st;
  if ((st = c->upload_refs(refs, f)) != PRNU_OK) return st;
  std::vector<CandParam> params((size_t)n, CandParam{0.f, 0.f, frame, 0});
  std::vector<CandRecord> recs;
  if ((st = c->evaluate(search_shape(f, frames, shift_radius), frames->dtype, params, recs, &proj)) != PRNU_OK) return st;
  for (int i = 0; i < n; ++i) {
    pce[i] = recs[(size_t)i].pce;
    if (rho) rho[i] = recs[(size_t)i].rho;
    if (dx) dx[i] = recs[(size_t)i].dx;
    if (dy) dy[i] = recs[(size_t)i].dy;
  }
  return PRNU_OK;
}

prnu_status prnu_search_with_transform(prnu_ctx* ctx, prnu_fp fp, const prnu_frames* frames,
                                       const prnu_search_opts* opts, const double* H, prnu_frame_result* out,
                                       prnu_video_summary* summary) {
  if (!ctx || !frames || !opts || (frames->n_frames > 0 && (!H || !out))) return fail(PRNU_E_ARG, "null argument");
  if (!opts->refine) return fail(PRNU_E_ARG, "the transform-initialised search runs the refinement (refine = 1)");
  Context* c = reinterpret_cast<Context*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->failed) return fail(PRNU_E_DEVICE, "context failed earlier");
  Fingerprint f;
  if (!c->get_fp(fp, f)) return fail(PRNU_E_HANDLE, "unknown fingerprint %llu", (unsigned long long)fp);
  prnu_status st = validate_opts(opts);
  if (st != PRNU_OK) return st;
  if ((st = validate_frames(frames, f, opts->shift_radius)) != PRNU_OK) return st;
  const int F = frames->n_frames;
  // per frame: the caller's transform, then the identity
  std::vector<float> proj((size_t)F * 18);
  const double I[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  for (int i = 0; i < F; ++i) {
    if (!transform_inverse(H + (size_t)i * 9, proj.data() + (size_t)i * 18))
      return fail(PRNU_E_ARG, "transform of frame %d is not finite or not invertible", i);
    (void)transform_inverse(I, proj.data() + (size_t)i * 18 + 9);
  }
  (void)hipSetDevice(c->device);
  if (F > 0) {
    std::vector<FrameRef> refs;
    if ((st = c->stage_frames(frames, refs)) != PRNU_OK) return st;
    if ((st = c->upload_refs(refs, f)) != PRNU_OK) return st;
    std::vector<CandParam> params;
    for (int i = 0; i < F; ++i) {
      params.push_back(CandParam{0.f, 0.f, i, 0});
      params.push_back(CandParam{0.f, 0.f, i, 0});
    }
    std::vector<CandRecord> recs;
    const Shape sh = search_shape(f, frames, opts->shift_radius);
    if ((st = c->evaluate(sh, frames->dtype, params, recs, &proj)) != PRNU_OK) return st;
    // Algorithm 1: start from the transform where it scores higher than the frame as is
    std::vector<std::pair<double, double>> inits((size_t)F);
    std::vector<int> used((size_t)F);
    for (int i = 0; i < F; ++i) {
      used[(size_t)i] = recs[(size_t)2 * i].pce > recs[(size_t)2 * i + 1].pce ? 1 : 0;
      inits[(size_t)i] = used[(size_t)i] ? similarity_of(H + (size_t)i * 9)
                                         : (opts->has_init ? std::make_pair(opts->init_scale, opts->init_rot_deg)
                                                           : std::make_pair(1.0, 0.0));
    }
    if ((st = c->refine(sh, frames->dtype, F, opts, inits, out)) != PRNU_OK) return st;
    for (int i = 0; i < F; ++i) out[i].used_init = used[(size_t)i];
  }
  if (summary) {
    double sum = 0.0;
    for (int i = 0; i < F; ++i) sum += out[i].pce;
    summary->n_frames = F;
    summary->mean_pce = F ? sum / F : 0.0;
    summary->decision = summary->mean_pce > opts->tau;
    summary->queue_s = 0.0;
    summary->latency_s = 0.0;
  }
  return PRNU_OK;
}

// Tight (L, M, N) fp32 device view of frames: the caller's buffer when it already is
// one (contiguous, 16-byte aligned, ordered after the caller's stream), else a copy.
static prnu_status tight_frames(Context& ctx, hipStream_t s, const prnu_frames* fr, DevBuf& buf, HostBuf& pinned,
                                const float** out) {
  const int M = fr->height, N = fr->width, L = fr->n_frames;
  const size_t fbytes = (size_t)M * N * sizeof(float);
  hipError_t e;
  if (fr->on_device) {
    prnu_status st = order_after(ctx, s, fr->stream);
    if (st != PRNU_OK) return st;
    if (fr->row_stride == N && (L == 1 || fr->frame_stride == (int64_t)M * N) &&
        ((uintptr_t)fr->data & 15) == 0) {
      *out = reinterpret_cast<const float*>(fr->data);
      return PRNU_OK;
    }
  }
  if ((e = buf.reserve(fbytes * (size_t)L)) != hipSuccess) return fail(PRNU_E_NOMEM, "image staging");
  const char* src = reinterpret_cast<const char*>(fr->data);
  if (!fr->on_device) {
    if ((e = upload_tight(s, src, sizeof(float), L, M, N, fr->frame_stride, fr->row_stride, pinned, buf.ptr)) !=
        hipSuccess)
      return staging_fail(ctx, e, "image staging");
  } else {
    for (int l = 0; l < L; ++l) {
      e = hipMemcpy2DAsync(reinterpret_cast<char*>(buf.ptr) + (size_t)l * fbytes, (size_t)N * sizeof(float),
                           src + (size_t)l * fr->frame_stride * sizeof(float), (size_t)fr->row_stride * sizeof(float),
                           (size_t)N * sizeof(float), (size_t)M, hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return ctx.hip_fail(e, "image staging");
    }
  }
  *out = reinterpret_cast<const float*>(buf.ptr);
  return PRNU_OK;
}

prnu_status prnu_estimate_fingerprint(prnu_ctx* ctx, const prnu_frames* images, const prnu_frames* residuals,
                                      float* K, int32_t out_on_device) {
  if (!ctx || !images || !residuals || !K) return fail(PRNU_E_ARG, "null argument");
  for (const prnu_frames* fr : {images, residuals}) {
    if (fr->dtype != PRNU_F32) return fail(PRNU_E_ARG, "images and residuals must be float32");
    if (fr->n_frames < 1 || !fr->data) return fail(PRNU_E_ARG, "no images");
    if (fr->height < 1 || fr->width < 1) return fail(PRNU_E_SHAPE, "empty image");
    if (fr->row_stride < fr->width) return fail(PRNU_E_ARG, "row stride smaller than the width");
    if (fr->n_frames > 1 && fr->frame_stride < fr->row_stride * fr->height) return fail(PRNU_E_ARG, "frame stride");
  }
  if (images->n_frames != residuals->n_frames || images->height != residuals->height ||
      images->width != residuals->width)
    return fail(PRNU_E_SHAPE, "images and residuals differ in count or size");
  Context* c = reinterpret_cast<Context*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->failed) return fail(PRNU_E_DEVICE, "context failed earlier");
  (void)hipSetDevice(c->device);
  hipStream_t s = c->runner.stream;
  DevBuf bi, bw, bk;
  HostBuf pi, pw;
  const float *I = nullptr, *W = nullptr;
  prnu_status st;
  if ((st = tight_frames(*c, s, images, bi, pi, &I)) != PRNU_OK) return st;
  if ((st = tight_frames(*c, s, residuals, bw, pw, &W)) != PRNU_OK) return st;
  const int64_t MN = (int64_t)images->height * images->width;
  hipError_t e;
  float* dk = K;
  if (!out_on_device) {
    if ((e = bk.reserve((size_t)MN * sizeof(float))) != hipSuccess) return fail(PRNU_E_NOMEM, "fingerprint output");
    dk = reinterpret_cast<float*>(bk.ptr);
  } else if (((uintptr_t)K & 15) != 0) {
    return fail(PRNU_E_ARG, "device output must be 16-byte aligned");
  }
  if ((e = launch_estimate_fp(I, W, images->n_frames, MN, dk, s)) != hipSuccess)
    return c->hip_fail(e, "fingerprint estimation");
  if (!out_on_device &&
      (e = hipMemcpyAsync(K, dk, (size_t)MN * sizeof(float), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return c->hip_fail(e, "fingerprint download");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return c->hip_fail(e, "fingerprint estimation");
  return PRNU_OK;
}

prnu_status prnu_extract_residuals(prnu_ctx* ctx, const prnu_frames* images, double sigma0, float* out,
                                   int32_t out_on_device) {
  if (!ctx || !images || (images->n_frames > 0 && (!out || !images->data))) return fail(PRNU_E_ARG, "null argument");
  if (images->dtype != PRNU_F32) return fail(PRNU_E_ARG, "images must be float32");
  if (images->n_frames < 0) return fail(PRNU_E_ARG, "negative image count");
  if (!(sigma0 >= 0.0) || !std::isfinite(sigma0)) return fail(PRNU_E_ARG, "sigma0 must be finite and >= 0");
  const int M = images->height, N = images->width, L = images->n_frames;
  // the mirrored extension to multiples of 16 needs at least 9 rows and columns
  if (M < 9 || N < 9) return fail(PRNU_E_SHAPE, "image %dx%d: residual extraction needs at least 9x9", M, N);
  if (images->row_stride < N) return fail(PRNU_E_ARG, "row stride smaller than the width");
  if (L > 1 && images->frame_stride < images->row_stride * M) return fail(PRNU_E_ARG, "frame stride");
  if (L == 0) return PRNU_OK;
  Context* c = reinterpret_cast<Context*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->failed) return fail(PRNU_E_DEVICE, "context failed earlier");
  (void)hipSetDevice(c->device);
  hipStream_t s = c->runner.stream;
  const size_t per = residual_workspace_floats(M, N), MN = (size_t)M * N;
  // images per pass: the workspace stays within 2 GiB
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)L, (2ull << 30) / (per * sizeof(float))));
  hipError_t e;
  if ((e = c->res_ws.reserve(per * sizeof(float) * (size_t)chunk)) != hipSuccess)
    return fail(PRNU_E_NOMEM, "residual workspace: %s", hipGetErrorString(e));
  if (images->on_device) {
    prnu_status st = order_after(*c, s, images->stream);
    if (st != PRNU_OK) return st;
  } else if ((e = c->res_in.reserve(MN * sizeof(float) * (size_t)chunk)) != hipSuccess) {
    return fail(PRNU_E_NOMEM, "image staging: %s", hipGetErrorString(e));
  }
  if (!out_on_device && (e = c->res_out.reserve(MN * sizeof(float) * (size_t)chunk)) != hipSuccess)
    return fail(PRNU_E_NOMEM, "residual staging: %s", hipGetErrorString(e));
  for (int l0 = 0; l0 < L; l0 += chunk) {
    const int n = std::min(chunk, L - l0);
    const float* in;
    int64_t is, rs;
    if (images->on_device) {
      in = reinterpret_cast<const float*>(images->data) + (int64_t)l0 * images->frame_stride;
      is = images->frame_stride, rs = images->row_stride;
    } else {
      const float* h = reinterpret_cast<const float*>(images->data) + (int64_t)l0 * images->frame_stride;
      if ((e = upload_tight(s, h, sizeof(float), n, M, N, images->frame_stride, images->row_stride, c->res_pinned,
                            c->res_in.ptr)) != hipSuccess)
        return staging_fail(*c, e, "image upload");
      in = reinterpret_cast<const float*>(c->res_in.ptr);
      is = (int64_t)MN, rs = N;
    }
    float* dst = out_on_device ? out + (size_t)l0 * MN : reinterpret_cast<float*>(c->res_out.ptr);
    if ((e = launch_residuals(in, is, rs, n, M, N, (float)sigma0, reinterpret_cast<float*>(c->res_ws.ptr), dst,
                              (int64_t)MN, N, s)) != hipSuccess)
      return c->hip_fail(e, "residual extraction");
    // to host memory through pinned memory (one DMA), then a host copy
    if (!out_on_device) {
      if ((e = c->res_pinned_out.reserve((size_t)chunk * MN * sizeof(float))) != hipSuccess)
        return fail(PRNU_E_NOMEM, "pinned residual staging: %s", hipGetErrorString(e));
      if ((e = hipMemcpyAsync(c->res_pinned_out.ptr, dst, (size_t)n * MN * sizeof(float), hipMemcpyDeviceToHost,
                              s)) != hipSuccess)
        return c->hip_fail(e, "residual download");
    }
    // the staging buffers are reused by the next pass
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return c->hip_fail(e, "residual extraction");
    if (!out_on_device) std::memcpy(out + (size_t)l0 * MN, c->res_pinned_out.ptr, (size_t)n * MN * sizeof(float));
  }
  return PRNU_OK;
}

prnu_status prnu_tune(prnu_ctx* ctx, int32_t height, int32_t width, int32_t shift_radius, prnu_dtype dtype,
                      int32_t* batch, int32_t* order, double* ns_per_candidate, int32_t* from_cache) {
  if (!ctx) return fail(PRNU_E_ARG, "null context");
  if (dtype != PRNU_F32 && dtype != PRNU_BF16) return fail(PRNU_E_ARG, "unknown dtype %d", (int)dtype);
  Context* c = reinterpret_cast<Context*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->failed) return fail(PRNU_E_DEVICE, "context failed earlier");
  prnu_status st = check_shape(height, width, shift_radius);
  if (st != PRNU_OK) return st;
  (void)hipSetDevice(c->device);
  Schedule sc;
  if ((st = c->schedule(Shape{height, width, shift_radius}, dtype, c->runner, sc)) != PRNU_OK) return st;
  if (batch) *batch = sc.chunk;
  if (order) *order = sc.order;
  if (ns_per_candidate) *ns_per_candidate = sc.ns_per_cand;
  if (from_cache) *from_cache = sc.from_cache ? 1 : 0;
  return PRNU_OK;
}

int32_t prnu_candidates(const prnu_search_opts* opts, int32_t kind, int32_t iteration, double cs, double ct,
                        double* out, int32_t cap) {
  if (!opts || cap < 0 || (cap > 0 && !out)) return fail(PRNU_E_ARG, "null argument");
  std::vector<Cand> list;
  switch (kind) {
    case 0:
      if (opts->full.n_scale < 1 || opts->full.n_rot < 1 || (long)opts->full.n_scale * opts->full.n_rot > (1L << 20))
        return fail(PRNU_E_ARG, "full grid size");
      full_candidates(opts->full, list);
      break;
    case 1:
      if (opts->local_n_scale < 1 || opts->local_n_rot < 1 ||
          (long)opts->local_n_scale * opts->local_n_rot > (1L << 20))
        return fail(PRNU_E_ARG, "local grid size");
      local_candidates(*opts, cs, ct, list);
      break;
    case 2: {
      if (iteration < 1 || iteration > 8) return fail(PRNU_E_ARG, "iteration %d", iteration);
      prnu_search_opts o = *opts;
      o.refine = 1;
      o.warm = 0;
      const prnu_status st = validate_opts(&o);
      if (st != PRNU_OK) return st;
      refine_candidates(o, iteration, cs, ct, list);
      break;
    }
    default: return fail(PRNU_E_ARG, "unknown grid kind %d", kind);
  }
  for (int i = 0; i < (int)list.size() && i < cap; ++i) {
    out[2 * i] = list[(size_t)i].scale;
    out[2 * i + 1] = list[(size_t)i].rot_deg;
  }
  return (int32_t)list.size();
}

prnu_status prnu_check_opts(const prnu_search_opts* opts) { return validate_opts(opts); }

prnu_status prnu_graph_stats(prnu_ctx* ctx, int64_t* captures, int64_t* replays) {
  if (!ctx) return fail(PRNU_E_ARG, "null context");
  Context* c = reinterpret_cast<Context*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  if (captures) *captures = c->runner.graph_captures;
  if (replays) *replays = c->runner.graph_replays;
  return PRNU_OK;
}

prnu_status prnu_profile_enable(prnu_ctx* ctx, int32_t enable) {
  if (!ctx) return fail(PRNU_E_ARG, "null context");
  Context* c = reinterpret_cast<Context*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  c->runner.prof_on = enable != 0;
  for (auto& p : c->runner.prof) p = KernelStat{};
  return PRNU_OK;
}

prnu_status prnu_profile_read(prnu_ctx* ctx, prnu_kernel_stats* out) {
  if (!ctx || !out) return fail(PRNU_E_ARG, "null argument");
  Context* c = reinterpret_cast<Context*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  static const char* names[PRNU_NUM_KERNELS] = {"warp_rowfft", "col_product", "band_rowifft", "pce"};
  for (int k = 0; k < PRNU_NUM_KERNELS; ++k) {
    out[k].name = names[k];
    out[k].launches = c->runner.prof[k].launches;
    out[k].total_ms = c->runner.prof[k].total_ms;
    out[k].candidates = c->runner.prof[k].candidates;
    out[k].algo_bytes = c->runner.prof[k].algo_bytes;
  }
  return PRNU_OK;
}

}  // extern "C"
