// Serving engine behind prnu_submit_video / prnu_poll / prnu_cancel: continuous
// batching of videos against device-resident fingerprints.
//
// Videos are copied into library-owned memory at submission and queued.  A worker
// thread admits queued videos while a slot is free and their device footprint (the
// zero-bordered frames) fits the HBM budget, uploads them on an upload stream, and then
// runs the chained search of every admitted video: each iteration takes the next
// candidate list of every ready video (full grid for a first frame, local grid around
// the previous estimate, or the full-grid fallback), groups the lists by frame shape,
// and issues one set of search launches per group, so that candidates of many videos
// share each launch.  Two such batches are kept in flight; the results of a finished
// batch advance the videos (argmax, fallback decision, next frame) while the next batch
// runs.  A finished video releases its slot and device memory and is returned by
// prnu_poll exactly once.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <tuple>

#include "runtime.hpp"

namespace prnu {

namespace {

enum VideoState { kQueued = 0, kActive = 1, kDone = 2 };
enum ItemKind { kFull = 0, kLocal = 1, kFallback = 2, kRefine = 3 };

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
  std::vector<float> scales;
  bool staged_at_submit = false;
  bool charged = false;  // footprint counted in the engine's used bytes
  size_t footprint = 0;
  hipEvent_t ready = nullptr;  // upload finished
  VideoState state = kQueued;
  prnu_status status = PRNU_OK;
  bool cancel = false;
  // search progress
  int frame = 0;
  bool in_flight = false;
  bool have_centre = false;
  double cs = 1.0, ct = 0.0;
  bool fallback_pending = false;
  int refine_iter = 0;             // refinement iterations done on the current frame
  double rcs = 1.0, rct = 0.0;     // the current frame's refinement estimate
  std::vector<Cand> list;          // candidates evaluated for the current frame
  std::vector<CandRecord> recs;    // their records
  std::vector<prnu_frame_result> results;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

struct Item {
  Video* v;
  int kind;
  int offset, n;
  std::vector<Cand> cands;
};

struct Launch {
  Shape sh;
  int dtype = 0;
  std::vector<Item> items;
  int n = 0;
  HostBuf h_cand, h_rec, h_refs;
  DevBuf d_cand, d_rec, d_frefs, d_fprefs;
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
  void finish_frame(Video* v, int best);
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

void ServingEngine::finish_frame(Video* v, int best) {
  prnu_frame_result& r = v->results[(size_t)v->frame];
  std::memset(&r, 0, sizeof(r));
  r.n_evaluated = (int)v->recs.size();
  r.fell_back = v->fallback_pending ? 1 : 0;
  r.iterations = v->opts.refine ? v->refine_iter : 0;
  if (best < 0) {
    r.status = PRNU_E_NONFINITE;
    r.pce = NAN;
  } else {
    fill_result(r, v->recs[(size_t)best], v->list[(size_t)best], best);
    v->have_centre = true;
    v->cs = v->list[(size_t)best].scale;
    v->ct = v->list[(size_t)best].rot_deg;
  }
  v->frame++;
  v->fallback_pending = false;
  v->refine_iter = 0;
  v->rcs = v->opts.has_init ? v->opts.init_scale : 1.0;
  v->rct = v->opts.has_init ? v->opts.init_rot_deg : 0.0;
  v->list.clear();
  v->recs.clear();
}

// Apply a finished batch's records to its videos (called with mu held).
void ServingEngine::complete(Launch& L) {
  const CandRecord* rec = reinterpret_cast<const CandRecord*>(L.h_rec.ptr);
  for (Item& it : L.items) {
    Video* v = it.v;
    v->in_flight = false;
    if (v->state != kActive) continue;
    v->list.insert(v->list.end(), it.cands.begin(), it.cands.end());
    v->recs.insert(v->recs.end(), rec + it.offset, rec + it.offset + it.n);
    const int best = argmax_records(v->recs.data(), (int)v->recs.size());
    if (it.kind == kRefine) {
      // move to this iteration's argmax; stop when it repeats or after the last iteration
      const int bi = argmax_records(rec + it.offset, it.n);
      ++v->refine_iter;
      bool stop = bi < 0 || v->refine_iter >= v->opts.refine_max_iter;
      if (bi >= 0) {
        const Cand& e = it.cands[(size_t)bi];
        if (e.scale == v->rcs && e.rot_deg == v->rct) stop = true;
        v->rcs = e.scale;
        v->rct = e.rot_deg;
      }
      if (stop) finish_frame(v, best);
    } else if (it.kind == kLocal && (best < 0 || !(v->recs[(size_t)best].pce >= v->opts.fallback_pce))) {
      v->fallback_pending = true;  // the full grid follows for this frame
    } else {
      finish_frame(v, best);
    }
    if (v->cancel)
      finalize(v, PRNU_E_CANCELLED);
    else if (v->frame >= v->F)
      finalize(v, PRNU_OK);
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
    int n = 0;
    for (Item* it : g.second) {
      it->offset = n;
      n += it->n;
    }
    L->n = n;
    const int slots_n = (int)g.second.size();
    hipError_t e;
    const size_t refb = sizeof(FrameRef) * (size_t)slots_n + sizeof(FpRef) * (size_t)slots_n;
    if ((e = L->h_cand.reserve(sizeof(CandParam) * (size_t)n)) != hipSuccess ||
        (e = L->h_rec.reserve(sizeof(CandRecord) * (size_t)n)) != hipSuccess ||
        (e = L->h_refs.reserve(refb)) != hipSuccess ||
        (e = L->d_cand.reserve(sizeof(CandParam) * (size_t)n)) != hipSuccess ||
        (e = L->d_rec.reserve(sizeof(CandRecord) * (size_t)n)) != hipSuccess ||
        (e = L->d_frefs.reserve(sizeof(FrameRef) * (size_t)slots_n)) != hipSuccess ||
        (e = L->d_fprefs.reserve(sizeof(FpRef) * (size_t)slots_n)) != hipSuccess ||
        (!L->done && (e = hipEventCreateWithFlags(&L->done, hipEventDisableTiming)) != hipSuccess)) {
      ctx.hip_fail(e, "serving batch buffers");
      throw std::runtime_error("device");
    }
    CandParam* hc = reinterpret_cast<CandParam*>(L->h_cand.ptr);
    FrameRef* hf = reinterpret_cast<FrameRef*>(L->h_refs.ptr);
    FpRef* hp = reinterpret_cast<FpRef*>(reinterpret_cast<char*>(L->h_refs.ptr) + sizeof(FrameRef) * (size_t)slots_n);
    for (int s = 0; s < slots_n; ++s) {
      Item* it = g.second[(size_t)s];
      Video* v = it->v;
      const size_t fbytes = (size_t)padded_frame(v->M, v->N) * v->esz;
      hf[s] = FrameRef{reinterpret_cast<const char*>(v->padded.ptr) + (size_t)v->frame * fbytes,
                       v->dtype == PRNU_BF16 ? reinterpret_cast<const float*>(v->dscales.ptr) + v->frame : nullptr};
      hp[s] = FpRef{v->fp.FK, v->fp.norm};
      for (int i = 0; i < it->n; ++i) hc[it->offset + i] = make_param(it->cands[(size_t)i], s, s);
      L->items.push_back(std::move(*it));
    }
    hipStream_t s = runner.stream;
    if ((e = hipMemcpyAsync(L->d_cand.ptr, hc, sizeof(CandParam) * (size_t)n, hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(L->d_frefs.ptr, hf, sizeof(FrameRef) * (size_t)slots_n, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(L->d_fprefs.ptr, hp, sizeof(FpRef) * (size_t)slots_n, hipMemcpyHostToDevice, s)) !=
            hipSuccess) {
      ctx.hip_fail(e, "serving batch upload");
      throw std::runtime_error("device");
    }
    prnu_status st = runner.run(ctx, L->sh, L->dtype, reinterpret_cast<FrameRef*>(L->d_frefs.ptr),
                                reinterpret_cast<FpRef*>(L->d_fprefs.ptr), reinterpret_cast<CandParam*>(L->d_cand.ptr),
                                reinterpret_cast<CandRecord*>(L->d_rec.ptr), n);
    if (st != PRNU_OK) throw std::runtime_error("device");
    if ((e = hipMemcpyAsync(L->h_rec.ptr, L->d_rec.ptr, sizeof(CandRecord) * (size_t)n, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
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
        // next work item of every ready, idle video
        for (Video* v : std::vector<Video*>(active)) {
          if (v->in_flight || v->frame >= v->F) continue;
          if (v->cancel) {
            finalize(v, PRNU_E_CANCELLED);
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
          const bool warm = v->opts.warm != 0;
          if (v->opts.refine) {
            it.kind = kRefine;
            refine_candidates(v->opts, v->refine_iter + 1, v->rcs, v->rct, it.cands);
          } else if (!warm || (!v->have_centre && !v->fallback_pending)) {
            it.kind = kFull;
            full_candidates(v->opts.full, it.cands);
          } else if (v->fallback_pending) {
            it.kind = kFallback;
            full_candidates(v->opts.full, it.cands);
          } else {
            it.kind = kLocal;
            local_candidates(v->opts, v->cs, v->ct, it.cands);
          }
          it.n = (int)it.cands.size();
          it.offset = 0;
          v->in_flight = true;
          items.push_back(std::move(it));
        }
        if (items.empty() && inflight.empty()) {
          // nothing to run: wait for submissions, uploads or cancellations
          cv_work.wait_for(lk, std::chrono::milliseconds(queued.empty() && active.empty() ? 50 : 1));
          continue;
        }
      }
      if (!items.empty()) build_and_launch(items);
      // Keep at most two batches in flight: complete the oldest when it is done (or
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
                 sizeof(float) * (size_t)std::max(1, v->F);
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
