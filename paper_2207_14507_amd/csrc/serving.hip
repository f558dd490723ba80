// Serving engine behind prnu_submit_video / prnu_poll / prnu_cancel: continuous
// batching of videos against device-resident fingerprints.
//
// Videos are copied into library-owned memory at submission and queued.  A worker
// thread admits queued videos while a slot is free and their device footprint (the
// zero-bordered frames and the chain state) fits the HBM budget, and uploads them on an
// upload stream.  Each iteration then takes one frame of every admitted video that can
// take one, groups the frames by shape, and issues one launch per group, so that
// candidates of many videos share each launch of the search kernels:
//   - a chained video (warm start, or every frame on the full grid) advances on the
//     device alone: its next frame's candidates come from the state its previous frame
//     left there, and the full-grid fallback is decided and searched on the device
//     (chain.hpp).  The host only counts finished frames, and keeps up to two frames of
//     such a video in flight;
//   - a video searched by the coarse-to-fine refinement takes one iteration per launch:
//     the device reduces the iteration's grid to its best candidate and the host reads
//     it back to place the next grid or stop the frame.
// A finished video's results are read back, its slot and device memory are released,
// and prnu_poll returns it exactly once.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <tuple>

#include "runtime.hpp"

namespace prnu {

namespace {

enum VideoState { kQueued = 0, kActive = 1, kDone = 2 };
enum ItemKind { kChained = 0, kRefineStep = 1 };

// Frames of one chained video allowed in flight at once (consecutive launches).
constexpr int kChainDepth = 2;

struct Video {
  prnu_ticket id = 0;
  prnu_fp fp_handle = 0;
  Fingerprint fp;
  prnu_search_opts opts{};
  int F = 0, M = 0, N = 0, dtype = 0;  // frame count and frame size (at most fp.M x fp.N)
  size_t esz = 4;
  // library-owned copy of the frames: pinned host (tight rows) or, for device input,
  // the zero-bordered device layout directly
  HostBuf host_copy;
  DevBuf tight, padded, dscales;
  DevBuf dchain;  // ChainState, FrameBest, then F result records
  std::vector<float> scales;
  bool staged_at_submit = false;
  bool charged = false;  // footprint counted in the engine's used bytes
  size_t footprint = 0;
  hipEvent_t ready = nullptr;  // upload finished
  VideoState state = kQueued;
  prnu_status status = PRNU_OK;
  bool cancel = false;
  int in_flight = 0;     // items of this video in launches not yet completed
  // chained videos: frames enqueued and frames whose launch has completed
  int next_frame = 0, done_frames = 0;
  bool recent_fallback = false;  // the last completed frame searched the full grid too
  // refined videos: the current frame, its iterations so far and its estimate
  int frame = 0;
  int refine_iter = 0;
  double rcs = 1.0, rct = 0.0;
  std::vector<prnu_frame_result> results;
  double t_submit = 0, t_admit = 0, t_done = 0;

  bool refined() const { return opts.refine != 0; }
  ChainState* dstate() { return reinterpret_cast<ChainState*>(dchain.ptr); }
  FrameBest* dbest() { return reinterpret_cast<FrameBest*>(reinterpret_cast<char*>(dchain.ptr) + 64); }
  prnu_frame_result* dres() { return reinterpret_cast<prnu_frame_result*>(reinterpret_cast<char*>(dchain.ptr) + 192); }
};
// dchain layout: ChainState at 0, FrameBest at 64, results from 192
static_assert(sizeof(ChainState) <= 64 && sizeof(FrameBest) <= 128, "chain layout");
size_t chain_bytes(int F) { return 192 + sizeof(prnu_frame_result) * (size_t)std::max(1, F); }

struct Item {
  Video* v;
  int kind;
  int frame;
  int iter;                    // refinement iteration (1-based)
  std::vector<CandSite> list;  // refinement grid
};

struct Launch {
  Shape sh;
  int dtype = 0;
  std::vector<Item> items;
  bool has_refine = false;
  HostBuf h_items, h_lists, h_refs, h_outs;
  DevBuf d_items, d_outs, d_cand, d_site, d_rec, d_fbc, d_fbs, d_fbr, d_ndev, d_lists, d_frefs, d_fprefs;
  hipEvent_t done = nullptr;
};

}  // namespace

struct ServingEngine {
  Context& ctx;
  hipStream_t up_stream = nullptr;
  Runner runner;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::map<prnu_ticket, std::unique_ptr<Video>> videos;
  std::deque<Video*> queued;
  std::vector<Video*> active;
  uint64_t used_bytes = 0;
  uint64_t budget;
  int slots;
  int max_queue = 1024;
  prnu_ticket next_ticket = 0;
  bool stop = false;
  std::deque<std::unique_ptr<Launch>> inflight;
  std::vector<std::unique_ptr<Launch>> spare;  // recycled launch buffers
  std::thread worker;

  explicit ServingEngine(Context& c) : ctx(c), budget(c.hbm_budget), slots(c.max_slots) {}
  prnu_status start();
  ~ServingEngine();
  void loop();
  bool admit_locked();
  void build_and_launch(std::vector<Item>& items);
  void complete(Launch& L);
  bool fetch_results(Video* v);
  void finalize(Video* v, prnu_status st);
  void fail_all(prnu_status st);
};

void ServingDeleter::operator()(ServingEngine* e) const { delete e; }

prnu_status ServingEngine::start() {
  hipError_t e;
  if ((e = hipStreamCreateWithFlags(&runner.stream, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&up_stream, hipStreamNonBlocking)) != hipSuccess)
    return ctx.hip_fail(e, "serving streams");
  runner.batch_override = ctx.runner.batch_override;
  runner.use_graphs = ctx.runner.use_graphs;
  worker = std::thread([this] { loop(); });
  return PRNU_OK;
}

ServingEngine::~ServingEngine() {
  {
    std::lock_guard<std::mutex> lk(mu);
    stop = true;
  }
  cv_work.notify_all();
  if (worker.joinable()) worker.join();
  (void)hipSetDevice(ctx.device);
  if (runner.stream) (void)hipStreamSynchronize(runner.stream);
  if (up_stream) (void)hipStreamSynchronize(up_stream);
  for (auto& L : inflight)
    if (L->done) (void)hipEventDestroy(L->done);
  for (auto& L : spare)
    if (L->done) (void)hipEventDestroy(L->done);
  for (auto& kv : videos) {
    if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
    if (kv.second->state != kDone) {
      std::lock_guard<std::mutex> lf(ctx.fp_mu);
      auto it = ctx.fps.find(kv.second->fp_handle);
      if (it != ctx.fps.end()) it->second.users--;
    }
  }
  if (runner.stream) (void)hipStreamDestroy(runner.stream);
  if (up_stream) (void)hipStreamDestroy(up_stream);
}

// Admit queued videos while a slot and the budget allow (called with mu held).
bool ServingEngine::admit_locked() {
  bool any = false;
  while (!queued.empty() && (int)active.size() < slots) {
    Video* v = queued.front();
    if (!v->staged_at_submit && used_bytes + v->footprint > budget && !active.empty()) break;
    queued.pop_front();
    if (v->cancel) {
      finalize(v, PRNU_E_CANCELLED);
      continue;
    }
    if (!v->staged_at_submit) {
      used_bytes += v->footprint;
      v->charged = true;
      // upload + zero-bordered staging on the upload stream
      prnu_frames fr{};
      fr.data = v->host_copy.ptr;
      fr.dtype = (prnu_dtype)v->dtype;
      fr.n_frames = v->F;
      fr.height = v->M;
      fr.width = v->N;
      fr.frame_stride = (int64_t)v->M * v->N;
      fr.row_stride = v->N;
      fr.on_device = 0;
      prnu_status st = stage_padded(ctx, up_stream, &fr, v->tight, v->padded);
      hipError_t e = hipSuccess;
      if (st == PRNU_OK && v->dtype == PRNU_BF16) {
        if ((e = v->dscales.reserve(sizeof(float) * (size_t)std::max(1, v->F))) == hipSuccess)
          e = hipMemcpyAsync(v->dscales.ptr, v->scales.data(), sizeof(float) * (size_t)v->F, hipMemcpyHostToDevice,
                             up_stream);
      }
      if (st == PRNU_OK && e == hipSuccess) e = v->dchain.reserve(chain_bytes(v->F));
      if (st == PRNU_OK && e == hipSuccess) e = hipEventRecord(v->ready, up_stream);
      if (st != PRNU_OK || e != hipSuccess) {
        finalize(v, st != PRNU_OK ? st : PRNU_E_DEVICE);
        continue;
      }
    }
    v->state = kActive;
    v->t_admit = now_s();
    active.push_back(v);
    any = true;
  }
  return any;
}

void ServingEngine::finalize(Video* v, prnu_status st) {
  v->state = kDone;
  v->status = st;
  v->t_done = now_s();
  if (v->t_admit == 0) v->t_admit = v->t_done;
  if (v->charged) used_bytes -= v->footprint;
  v->charged = false;
  v->padded.release();
  v->tight.release();
  v->dscales.release();
  v->dchain.release();
  v->host_copy.release();
  active.erase(std::remove(active.begin(), active.end(), v), active.end());
  {
    std::lock_guard<std::mutex> lf(ctx.fp_mu);
    auto it = ctx.fps.find(v->fp_handle);
    if (it != ctx.fps.end()) it->second.users--;
  }
  cv_done.notify_all();
}

void ServingEngine::fail_all(prnu_status st) {
  std::lock_guard<std::mutex> lk(mu);
  while (!queued.empty()) {
    Video* v = queued.front();
    queued.pop_front();
    finalize(v, st);
  }
  while (!active.empty()) finalize(active.back(), st);
  stop = true;
  cv_done.notify_all();
}

// The video's results, written on the device by its launches (all completed), into
// v->results: a copy on the upload stream, so that launches in flight on the search
// stream are not waited for.
bool ServingEngine::fetch_results(Video* v) {
  HostBuf h;
  const size_t bytes = sizeof(prnu_frame_result) * (size_t)v->F;
  hipError_t e;
  if ((e = h.reserve(bytes)) != hipSuccess ||
      (e = hipMemcpyAsync(h.ptr, v->dres(), bytes, hipMemcpyDeviceToHost, up_stream)) != hipSuccess ||
      (e = hipStreamSynchronize(up_stream)) != hipSuccess) {
    ctx.hip_fail(e, "result download");
    return false;
  }
  std::memcpy(v->results.data(), h.ptr, bytes);
  return true;
}

// Apply a finished launch to its videos (called with mu held).
void ServingEngine::complete(Launch& L) {
  const ItemOut* outs = reinterpret_cast<const ItemOut*>(L.h_outs.ptr);
  for (size_t i = 0; i < L.items.size(); ++i) {
    Item& it = L.items[i];
    Video* v = it.v;
    v->in_flight--;
    if (v->state != kActive) continue;
    bool video_done = false;
    if (it.kind == kChained) {
      v->done_frames++;
      v->recent_fallback = outs[i].need != 0;
      video_done = v->done_frames >= v->F;
    } else {
      // move to this iteration's best; stop the frame when it repeats or after the last
      // iteration
      const ItemOut& o = outs[i];
      ++v->refine_iter;
      bool stop = o.seg_index < 0 || v->refine_iter >= v->opts.refine_max_iter;
      if (o.seg_index >= 0) {
        if (o.seg_s == v->rcs && o.seg_t == v->rct) stop = true;
        v->rcs = o.seg_s;
        v->rct = o.seg_t;
      }
      if (stop) {
        v->frame++;
        v->refine_iter = 0;
        v->rcs = v->opts.has_init ? v->opts.init_scale : 1.0;
        v->rct = v->opts.has_init ? v->opts.init_rot_deg : 0.0;
      }
      video_done = v->frame >= v->F;
    }
    if (v->in_flight > 0) continue;
    if (v->cancel) {
      finalize(v, PRNU_E_CANCELLED);
    } else if (video_done) {
      if (!fetch_results(v)) throw std::runtime_error("device");
      finalize(v, PRNU_OK);
    }
  }
  cv_work.notify_all();
}

// One launch per shape group: candidates of many videos share the kernels.
void ServingEngine::build_and_launch(std::vector<Item>& items) {
  // group by (transform size, frame size, radius, dtype)
  std::map<std::tuple<int, int, int, int, int, int>, std::vector<Item*>> groups;
  for (Item& it : items)
    groups[std::make_tuple(it.v->fp.M, it.v->fp.N, it.v->M, it.v->N, it.v->opts.shift_radius, it.v->dtype)].push_back(
        &it);
  for (auto& g : groups) {
    std::unique_ptr<Launch> L;
    if (!spare.empty()) {
      L = std::move(spare.back());
      spare.pop_back();
    } else {
      L.reset(new Launch());
    }
    L->items.clear();
    L->sh = Shape{std::get<0>(g.first), std::get<1>(g.first), std::get<4>(g.first)};
    L->sh.ey = std::get<0>(g.first) - std::get<2>(g.first);
    L->sh.ex = std::get<1>(g.first) - std::get<3>(g.first);
    L->dtype = std::get<5>(g.first);
    const int ni = (int)g.second.size();
    // candidate list, fallback list and refinement grids, in item order
    std::vector<ItemDesc> desc((size_t)ni);
    int n_total = 0, max_n = 0, max_fb = 0, fb_expect = 0;
    size_t n_sites = 0;
    std::vector<size_t> list_off((size_t)ni, 0);
    for (int k = 0; k < ni; ++k) {
      Item* it = g.second[(size_t)k];
      Video* v = it->v;
      const prnu_search_opts& o = v->opts;
      ItemDesc& d = desc[(size_t)k];
      d = ItemDesc{};
      d.slot = k;
      d.fslot = k;
      d.best = v->dbest();
      if (it->kind == kRefineStep) {
        d.gen.kind = kGenList;
        d.n = (int)it->list.size();
        d.mode = kModeRefine;
        d.merge = it->iter > 1;
        d.iter = it->iter;
        d.result = v->dres() + it->frame;
        list_off[(size_t)k] = n_sites;
        n_sites += it->list.size();
      } else {
        const int nf = o.full.n_scale * o.full.n_rot;
        d.result = v->dres() + it->frame;
        if (o.warm && (it->frame > 0 || o.has_init)) {
          d.gen = local_gen(o, v->dstate());
          d.n = o.local_n_scale * o.local_n_rot;
          d.full = full_gen(o.full);
          d.fb_n = nf;
          d.fallback_pce = o.fallback_pce;
          d.mode = kModeWarm;
          d.state = v->dstate();
          max_fb += nf;
          if (v->recent_fallback) fb_expect += nf;
        } else {
          d.gen = full_gen(o.full);
          d.n = nf;
          d.mode = kModePlain;
          d.state = o.warm ? v->dstate() : nullptr;
        }
      }
      d.off = n_total;
      n_total += d.n;
      max_n = std::max(max_n, d.n);
    }
    hipError_t e;
    const size_t refb = sizeof(FrameRef) * (size_t)ni + sizeof(FpRef) * (size_t)ni;
    const size_t nt = (size_t)std::max(1, n_total), nb = (size_t)std::max(1, max_fb), ns = std::max<size_t>(1, n_sites);
    if ((e = L->h_items.reserve(sizeof(ItemDesc) * (size_t)ni)) != hipSuccess ||
        (e = L->h_lists.reserve(sizeof(CandSite) * ns)) != hipSuccess ||
        (e = L->h_refs.reserve(refb)) != hipSuccess ||
        (e = L->h_outs.reserve(sizeof(ItemOut) * (size_t)ni)) != hipSuccess ||
        (e = L->d_items.reserve(sizeof(ItemDesc) * (size_t)ni)) != hipSuccess ||
        (e = L->d_outs.reserve(sizeof(ItemOut) * (size_t)ni)) != hipSuccess ||
        (e = L->d_cand.reserve(sizeof(CandParam) * nt)) != hipSuccess ||
        (e = L->d_site.reserve(sizeof(CandSite) * nt)) != hipSuccess ||
        (e = L->d_rec.reserve(sizeof(CandRecord) * nt)) != hipSuccess ||
        (e = L->d_fbc.reserve(sizeof(CandParam) * nb)) != hipSuccess ||
        (e = L->d_fbs.reserve(sizeof(CandSite) * nb)) != hipSuccess ||
        (e = L->d_fbr.reserve(sizeof(CandRecord) * nb)) != hipSuccess ||
        (e = L->d_ndev.reserve(sizeof(int))) != hipSuccess ||
        (e = L->d_lists.reserve(sizeof(CandSite) * ns)) != hipSuccess ||
        (e = L->d_frefs.reserve(sizeof(FrameRef) * (size_t)ni)) != hipSuccess ||
        (e = L->d_fprefs.reserve(sizeof(FpRef) * (size_t)ni)) != hipSuccess ||
        (!L->done && (e = hipEventCreateWithFlags(&L->done, hipEventDisableTiming)) != hipSuccess)) {
      ctx.hip_fail(e, "serving batch buffers");
      throw std::runtime_error("device");
    }
    ItemDesc* hi = reinterpret_cast<ItemDesc*>(L->h_items.ptr);
    CandSite* hl = reinterpret_cast<CandSite*>(L->h_lists.ptr);
    FrameRef* hf = reinterpret_cast<FrameRef*>(L->h_refs.ptr);
    FpRef* hp = reinterpret_cast<FpRef*>(reinterpret_cast<char*>(L->h_refs.ptr) + sizeof(FrameRef) * (size_t)ni);
    const CandSite* dl = reinterpret_cast<const CandSite*>(L->d_lists.ptr);
    L->has_refine = false;
    hipStream_t s = runner.stream;
    for (int k = 0; k < ni; ++k) {
      Item* it = g.second[(size_t)k];
      Video* v = it->v;
      const size_t fbytes = (size_t)padded_frame(v->M, v->N) * v->esz;
      hf[k] = FrameRef{reinterpret_cast<const char*>(v->padded.ptr) + (size_t)it->frame * fbytes,
                       v->dtype == PRNU_BF16 ? reinterpret_cast<const float*>(v->dscales.ptr) + it->frame : nullptr};
      hp[k] = FpRef{v->fp.FK, v->fp.norm};
      if (it->kind == kRefineStep) {
        desc[(size_t)k].gen.list = dl + list_off[(size_t)k];
        std::memcpy(hl + list_off[(size_t)k], it->list.data(), sizeof(CandSite) * it->list.size());
        L->has_refine = true;
      } else if (it->frame == 0) {
        // a chained video's first frame: its state starts from the initial transform
        const prnu_search_opts& o = v->opts;
        if ((e = launch_chain_init(v->dstate(), o.has_init, o.has_init ? o.init_scale : 1.0,
                                   o.has_init ? o.init_rot_deg : 0.0, s)) != hipSuccess) {
          ctx.hip_fail(e, "chain state");
          throw std::runtime_error("device");
        }
      }
      hi[k] = desc[(size_t)k];
      L->items.push_back(std::move(*it));
    }
    if ((e = hipMemcpyAsync(L->d_items.ptr, hi, sizeof(ItemDesc) * (size_t)ni, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (n_sites > 0 &&
         (e = hipMemcpyAsync(L->d_lists.ptr, hl, sizeof(CandSite) * n_sites, hipMemcpyHostToDevice, s)) != hipSuccess) ||
        (e = hipMemcpyAsync(L->d_frefs.ptr, hf, sizeof(FrameRef) * (size_t)ni, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(L->d_fprefs.ptr, hp, sizeof(FpRef) * (size_t)ni, hipMemcpyHostToDevice, s)) != hipSuccess) {
      ctx.hip_fail(e, "serving batch upload");
      throw std::runtime_error("device");
    }
    StepDev d;
    d.items = reinterpret_cast<const ItemDesc*>(L->d_items.ptr);
    d.outs = reinterpret_cast<ItemOut*>(L->d_outs.ptr);
    d.n_items = ni;
    d.cand = reinterpret_cast<CandParam*>(L->d_cand.ptr);
    d.site = reinterpret_cast<CandSite*>(L->d_site.ptr);
    d.rec = reinterpret_cast<CandRecord*>(L->d_rec.ptr);
    d.n_total = n_total;
    d.max_n = max_n;
    d.fb_cand = reinterpret_cast<CandParam*>(L->d_fbc.ptr);
    d.fb_site = reinterpret_cast<CandSite*>(L->d_fbs.ptr);
    d.fb_rec = reinterpret_cast<CandRecord*>(L->d_fbr.ptr);
    d.n_dev = reinterpret_cast<int*>(L->d_ndev.ptr);
    d.max_fb = max_fb;
    d.fb_expect = fb_expect;
    prnu_status st = runner.step(ctx, L->sh, L->dtype, reinterpret_cast<FrameRef*>(L->d_frefs.ptr),
                                 reinterpret_cast<FpRef*>(L->d_fprefs.ptr), d);
    if (st != PRNU_OK) throw std::runtime_error("device");
    // the items' outcomes come back with the launch: the next refinement centres, and
    // which warm frames fell back (the launch shape of later fallback chunks)
    if ((e = hipMemcpyAsync(L->h_outs.ptr, L->d_outs.ptr, sizeof(ItemOut) * (size_t)ni, hipMemcpyDeviceToHost,
                            s)) != hipSuccess ||
        (e = hipEventRecord(L->done, s)) != hipSuccess) {
      ctx.hip_fail(e, "serving batch");
      throw std::runtime_error("device");
    }
    inflight.push_back(std::move(L));
  }
}

void ServingEngine::loop() {
  (void)hipSetDevice(ctx.device);
  try {
    while (true) {
      std::vector<Item> items;
      {
        std::unique_lock<std::mutex> lk(mu);
        if (stop) break;
        // a device failure anywhere on the context (here or in a synchronous call)
        // ends every video
        if (ctx.failed) throw std::runtime_error("device");
        admit_locked();
        // next work item of every ready video that can take one
        for (Video* v : std::vector<Video*>(active)) {
          if (v->cancel) {
            if (v->in_flight == 0) finalize(v, PRNU_E_CANCELLED);
            continue;
          }
          if (!v->staged_at_submit) {
            const hipError_t q = hipEventQuery(v->ready);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
              ctx.hip_fail(q, "video upload");
              throw std::runtime_error("device");
            }
          }
          Item it;
          it.v = v;
          it.iter = 0;
          if (v->refined()) {
            if (v->in_flight > 0 || v->frame >= v->F) continue;
            it.kind = kRefineStep;
            it.frame = v->frame;
            it.iter = v->refine_iter + 1;
            std::vector<Cand> grid;
            refine_candidates(v->opts, it.iter, v->rcs, v->rct, grid);
            it.list.reserve(grid.size());
            for (const Cand& c : grid) it.list.push_back(CandSite{c.scale, c.rot_deg});
          } else {
            if (v->in_flight >= kChainDepth || v->next_frame >= v->F) continue;
            it.kind = kChained;
            it.frame = v->next_frame++;
          }
          v->in_flight++;
          items.push_back(std::move(it));
        }
        if (items.empty() && inflight.empty()) {
          // nothing to run: wait for submissions, uploads or cancellations
          cv_work.wait_for(lk, std::chrono::milliseconds(queued.empty() && active.empty() ? 50 : 1));
          continue;
        }
      }
      if (!items.empty()) build_and_launch(items);
      // Keep at most two launches in flight: complete the oldest when it is done (or
      // wait for it when the pipeline is full or there was nothing new to launch).
      while (!inflight.empty()) {
        Launch& L = *inflight.front();
        hipError_t q = hipEventQuery(L.done);
        if (q == hipErrorNotReady && (inflight.size() >= 2 || items.empty())) q = hipEventSynchronize(L.done);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) {
          ctx.hip_fail(q, "serving batch");
          throw std::runtime_error("device");
        }
        {
          std::lock_guard<std::mutex> lk(mu);
          complete(L);
        }
        spare.push_back(std::move(inflight.front()));
        inflight.pop_front();
        if (!items.empty()) break;  // launch the next batch before draining further
      }
    }
  } catch (const std::exception&) {
    fail_all(PRNU_E_DEVICE);
  }
}

ServingEngine* Context::engine() {
  if (!serving) {
    ServingEngine* e = new ServingEngine(*this);
    if (e->start() != PRNU_OK) {
      delete e;
      return nullptr;
    }
    serving.reset(e);
  }
  return serving.get();
}

void Context::shutdown_serving() { serving.reset(); }

}  // namespace prnu

using namespace prnu;

extern "C" {

prnu_status prnu_submit_video(prnu_ctx* ctx, prnu_fp fp, const prnu_frames* frames, const prnu_search_opts* opts,
                              prnu_ticket* out) {
  if (!ctx || !frames || !opts || !out) return fail(PRNU_E_ARG, "null argument");
  Context* c = reinterpret_cast<Context*>(ctx);
  if (c->failed) return fail(PRNU_E_DEVICE, "context failed earlier");
  Fingerprint f;
  if (!c->get_fp(fp, f)) return fail(PRNU_E_HANDLE, "unknown fingerprint %llu", (unsigned long long)fp);
  prnu_status st = validate_opts(opts);
  if (st != PRNU_OK) return st;
  if ((st = validate_frames(frames, f, opts->shift_radius)) != PRNU_OK) return st;
  (void)hipSetDevice(c->device);
  ServingEngine* E;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    E = c->engine();
  }
  if (!E) return fail(PRNU_E_DEVICE, "serving engine could not start");
  std::unique_ptr<Video> v(new Video());
  v->fp_handle = fp;
  v->fp = f;
  v->opts = *opts;
  v->rcs = opts->has_init ? opts->init_scale : 1.0;
  v->rct = opts->has_init ? opts->init_rot_deg : 0.0;
  v->F = frames->n_frames;
  v->M = frames->height;
  v->N = frames->width;
  v->dtype = frames->dtype;
  v->esz = frames->dtype == PRNU_BF16 ? 2 : 4;
  v->results.resize((size_t)std::max(1, v->F));
  v->footprint = (size_t)padded_frame(v->M, v->N) * v->esz * (size_t)std::max(1, v->F) +
                 sizeof(float) * (size_t)std::max(1, v->F) + chain_bytes(v->F);
  if (v->footprint > E->budget) return fail(PRNU_E_NOMEM, "video needs %zu bytes, budget is %llu", v->footprint,
                                            (unsigned long long)E->budget);
  hipError_t e;
  if ((e = hipEventCreateWithFlags(&v->ready, hipEventDisableTiming)) != hipSuccess)
    return c->hip_fail(e, "event create");
  {
    std::lock_guard<std::mutex> lk(E->mu);
    if ((int)E->queued.size() >= E->max_queue) {
      (void)hipEventDestroy(v->ready);
      return fail(PRNU_E_BUSY, "submission queue full");
    }
  }
  if (frames->on_device) {
    // Device input: stage straight into the zero-bordered device layout now (the
    // caller may free its buffer on return); charged to the budget immediately.
    {
      std::lock_guard<std::mutex> lk(E->mu);
      if (E->used_bytes + v->footprint > E->budget) {
        (void)hipEventDestroy(v->ready);
        return fail(PRNU_E_BUSY, "HBM budget in use; retry later");
      }
      E->used_bytes += v->footprint;
    }
    v->staged_at_submit = true;
    v->charged = true;
    DevBuf tmp;
    st = stage_padded(*c, E->up_stream, frames, tmp, v->padded);
    if (st == PRNU_OK && v->dtype == PRNU_BF16) {
      if ((e = v->dscales.reserve(sizeof(float) * (size_t)std::max(1, v->F))) != hipSuccess ||
          (v->F > 0 && (e = hipMemcpyAsync(v->dscales.ptr, frames->frame_scale, sizeof(float) * (size_t)v->F,
                                           hipMemcpyDeviceToDevice, E->up_stream)) != hipSuccess))
        st = c->hip_fail(e, "scale staging");
    }
    if (st == PRNU_OK && (e = v->dchain.reserve(chain_bytes(v->F))) != hipSuccess)
      st = fail(PRNU_E_NOMEM, "chain state: %s", hipGetErrorString(e));
    if (st == PRNU_OK && (e = hipStreamSynchronize(E->up_stream)) != hipSuccess) st = c->hip_fail(e, "staging");
    if (st != PRNU_OK) {
      std::lock_guard<std::mutex> lk(E->mu);
      E->used_bytes -= v->footprint;
      (void)hipEventDestroy(v->ready);
      return st;
    }
  } else {
    const size_t fbytes = (size_t)v->M * v->N * v->esz;
    if ((e = v->host_copy.reserve(fbytes * (size_t)std::max(1, v->F))) != hipSuccess) {
      (void)hipEventDestroy(v->ready);
      return fail(PRNU_E_NOMEM, "pinned staging for %zu bytes", fbytes * (size_t)v->F);
    }
    const char* src = reinterpret_cast<const char*>(frames->data);
    char* dst = reinterpret_cast<char*>(v->host_copy.ptr);
    for (int fi = 0; fi < v->F; ++fi)
      for (int y = 0; y < v->M; ++y)
        std::memcpy(dst + (size_t)fi * fbytes + (size_t)y * v->N * v->esz,
                    src + ((size_t)fi * frames->frame_stride + (size_t)y * frames->row_stride) * v->esz,
                    (size_t)v->N * v->esz);
    if (v->dtype == PRNU_BF16) v->scales.assign(frames->frame_scale, frames->frame_scale + v->F);
  }
  v->t_submit = now_s();
  {
    std::lock_guard<std::mutex> lf(c->fp_mu);
    auto it = c->fps.find(fp);
    if (it == c->fps.end()) {
      (void)hipEventDestroy(v->ready);
      return fail(PRNU_E_HANDLE, "fingerprint closed during submission");
    }
    it->second.users++;
  }
  std::lock_guard<std::mutex> lk(E->mu);
  if (E->stop) {
    // The engine ended on a device failure after this call's first check: nothing
    // would run the video.  Undo the charge and the fingerprint reference (mu before
    // fp_mu, the order finalize takes them in).
    if (v->charged) E->used_bytes -= v->footprint;
    (void)hipEventDestroy(v->ready);
    std::lock_guard<std::mutex> lf(c->fp_mu);
    auto it = c->fps.find(fp);
    if (it != c->fps.end()) it->second.users--;
    return fail(PRNU_E_DEVICE, "serving engine stopped after a device failure");
  }
  v->id = ++E->next_ticket;
  *out = v->id;
  Video* raw = v.get();
  E->videos[v->id] = std::move(v);
  if (raw->F == 0) {
    raw->t_admit = raw->t_submit;
    if (raw->charged) E->used_bytes -= raw->footprint;
    raw->charged = false;
    raw->state = kDone;
    raw->status = PRNU_OK;
    raw->t_done = now_s();
    std::lock_guard<std::mutex> lf(c->fp_mu);
    c->fps[fp].users--;
  } else {
    E->queued.push_back(raw);
  }
  E->cv_work.notify_all();
  return PRNU_OK;
}

prnu_status prnu_poll(prnu_ctx* ctx, prnu_ticket t, int32_t timeout_ms, prnu_frame_result* out,
                      prnu_video_summary* summary) {
  if (!ctx) return fail(PRNU_E_ARG, "null argument");
  Context* c = reinterpret_cast<Context*>(ctx);
  ServingEngine* E = c->serving.get();
  if (!E) return fail(PRNU_E_HANDLE, "unknown ticket %llu", (unsigned long long)t);
  std::unique_lock<std::mutex> lk(E->mu);
  auto it = E->videos.find(t);
  if (it == E->videos.end()) return fail(PRNU_E_HANDLE, "unknown ticket %llu", (unsigned long long)t);
  Video* v = it->second.get();
  // an engine that stopped has finished every video it held; the stop test only guards
  // against waiting on one it could no longer run
  auto done = [&] { return v->state == kDone || E->stop; };
  if (timeout_ms < 0)
    E->cv_done.wait(lk, done);
  else if (!E->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done))
    return PRNU_PENDING;
  if (v->state != kDone) return fail(PRNU_E_DEVICE, "serving engine stopped");
  const prnu_status st = v->status;
  if (out && v->F > 0) std::memcpy(out, v->results.data(), sizeof(prnu_frame_result) * (size_t)v->F);
  if (summary) {
    double s = 0.0;
    for (int f = 0; f < v->F; ++f) s += v->results[(size_t)f].pce;
    summary->n_frames = v->F;
    summary->mean_pce = v->F ? s / v->F : 0.0;
    summary->decision = summary->mean_pce > v->opts.tau;
    summary->queue_s = v->t_admit - v->t_submit;
    summary->latency_s = v->t_done - v->t_submit;
  }
  if (v->ready) (void)hipEventDestroy(v->ready);
  E->videos.erase(it);
  if (st != PRNU_OK) return fail(st, "video %llu ended with status %d", (unsigned long long)t, (int)st);
  return PRNU_OK;
}

prnu_status prnu_cancel(prnu_ctx* ctx, prnu_ticket t) {
  if (!ctx) return fail(PRNU_E_ARG, "null argument");
  Context* c = reinterpret_cast<Context*>(ctx);
  ServingEngine* E = c->serving.get();
  if (!E) return fail(PRNU_E_HANDLE, "unknown ticket %llu", (unsigned long long)t);
  std::lock_guard<std::mutex> lk(E->mu);
  auto it = E->videos.find(t);
  if (it == E->videos.end()) return fail(PRNU_E_HANDLE, "unknown ticket %llu", (unsigned long long)t);
  Video* v = it->second.get();
  if (v->state == kDone) return PRNU_OK;
  v->cancel = true;
  if (v->state == kQueued) {
    E->queued.erase(std::remove(E->queued.begin(), E->queued.end(), v), E->queued.end());
    E->finalize(v, PRNU_E_CANCELLED);
  }
  E->cv_work.notify_all();
  return PRNU_OK;
}

}  // extern "C"
