// Internal declarations of the host runtime.
#pragma once

#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/prnu.h"
#include "chain.hpp"
#include "kernels.hpp"

namespace prnu {

prnu_status fail(prnu_status s, const char* fmt, ...);

struct DevBuf {
  void* ptr = nullptr;
  size_t cap = 0;
  hipError_t reserve(size_t n);
  void release();
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
};

struct HostBuf {
  void* ptr = nullptr;
  size_t cap = 0;
  hipError_t reserve(size_t n);
  void release();
  HostBuf() = default;
  HostBuf(const HostBuf&) = delete;
  HostBuf& operator=(const HostBuf&) = delete;
  ~HostBuf() { release(); }
};

struct Fingerprint {
  int M = 0, N = 0;
  c32* FK = nullptr;  // column DFT of the packed half spectrum of K - mean, strip-tiled
  double mean = 0.0, norm = 0.0;
  int users = 0;      // videos in the serving engine that reference it
};

struct Cand {
  double scale, rot_deg;
};

struct KernelStat {
  int64_t launches = 0;
  double total_ms = 0.0;
  int64_t candidates = 0;
  double algo_bytes = 0.0;
};

struct ProfEvent {
  int kernel;
  hipEvent_t start, stop;
  int cands;
  double bytes;
};

// Grids and candidate generation (FP64, exactly centre + (k - (n-1)/2) * step).
double grid_node(int k, int n, double lo, double hi);
double local_node(int k, int n, double centre, double step);
void full_candidates(const prnu_grid& g, std::vector<Cand>& out);
void local_candidates(const prnu_search_opts& o, double cs, double ct, std::vector<Cand>& out);
void refine_candidates(const prnu_search_opts& o, int n, double cs, double ct, std::vector<Cand>& out);
CandParam make_param(const Cand& c, int frame, int fp);
prnu_status check_shape(int M, int N, int radius);
bool transform_inverse(const double* T, float* G);
std::pair<double, double> similarity_of(const double* T);
prnu_status validate_opts(const prnu_search_opts* o);
// Frame checks against the fingerprint and the shift radius: frames of the fingerprint's
// size or smaller (zero-padded), with at least 2R + 11 rows and columns.
prnu_status validate_frames(const prnu_frames* fr, const Fingerprint& fp, int radius);
// The search shape of frames against a fingerprint (transform size and padding).
Shape search_shape(const Fingerprint& fp, const prnu_frames* fr, int radius);
// Device grid descriptions of the full grid of opts and of the local grid around the
// centre held in *centre.
GridGen full_gen(const prnu_grid& g);
GridGen local_gen(const prnu_search_opts& o, const ChainState* centre);
double now_s();

class Context;

// Launch schedule of one problem shape: candidates per launch set (FFT batch) and the
// block order of the row and column kernels (Batch::order).
struct Schedule {
  int chunk = 0;
  int order = 0;
  double ns_per_cand = 0.0;  // measured by the tuner (0: default, untuned)
  bool from_cache = false;
};
using ShapeKey = std::tuple<int, int, int, int>;  // M, N, radius, dtype

// A captured launch set and the exact arguments it was captured with.
struct GraphEntry {
  std::vector<uintptr_t> key;
  hipGraphExec_t exec = nullptr;
  uint64_t last_use = 0;
};

// One launch of items (see chain.hpp), all arrays on the device: items[n_items] and
// their outputs; the candidate list (n_total entries, the longest item max_n) with its
// sites and records; the fallback list (max_fb entries at most, 0 when no item is warm)
// and its device-written length n_dev.
struct StepDev {
  const ItemDesc* items = nullptr;
  ItemOut* outs = nullptr;
  int n_items = 0;
  CandParam* cand = nullptr;
  CandSite* site = nullptr;
  CandRecord* rec = nullptr;
  int n_total = 0, max_n = 0;
  CandParam* fb_cand = nullptr;
  CandSite* fb_site = nullptr;
  CandRecord* fb_rec = nullptr;
  int* n_dev = nullptr;
  int max_fb = 0;
  // fallback candidates expected (from the items' previous frames): the chunks that
  // start below this are launched one workgroup per tile
  int fb_expect = 0;
};

// Launches the search kernels over candidate arrays already on the device, in chunks
// that fit its workspace, on one stream.  Optionally records per-kernel HIP events.
struct Runner {
  hipStream_t stream = nullptr;
  DevBuf ws_inter, ws_band, ws_win, ws_norm, ws_energy;
  double batch_bytes = 512.0 * 1024 * 1024;
  int batch_override = 0;
  bool prof_on = false;
  KernelStat prof[PRNU_NUM_KERNELS];
  std::vector<ProfEvent> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  bool use_graphs = true;
  std::vector<GraphEntry> graphs;  // captured launch sets, at most kMaxGraphs (LRU)
  std::vector<std::vector<uintptr_t>> seen;  // launch sets run once, not yet captured
  uint64_t graph_clock = 0;
  int64_t graph_replays = 0, graph_captures = 0;
  static constexpr size_t kMaxGraphs = 64, kMaxSeen = 64;

  ~Runner();
  int batch_size(const Shape& sh) const;
  // Launch set of candidates [0, n) in FFT batches of sc.chunk (no timing, no graph).
  hipError_t launch_all(const Shape& sh, int dtype, const FrameRef* frames, const FpRef* fps, const CandParam* cand,
                        const float* proj, CandRecord* rec, int n, const Schedule& sc, const c32* twM,
                        const c32* twMi, const c32* twN);
  void drop_graphs();
  size_t workspace_bytes(const Shape& sh, int nc) const;
  prnu_status ensure_workspace(const Shape& sh, int nc);
  // Candidates [0, n) of cand (device) with records to rec (device); proj (device, 9
  // floats per candidate, or null) selects the general Eq. (4) form.
  prnu_status run(Context& ctx, const Shape& sh, int dtype, const FrameRef* frames, const FpRef* fps,
                  const CandParam* cand, CandRecord* rec, int n, const float* proj = nullptr);
  // The same kernels over the first *n_dev (device-written, at most n_max) candidates:
  // device-counted launches in chunks of the schedule's batch.
  prnu_status run_dyn(Context& ctx, const Shape& sh, int dtype, const FrameRef* frames, const FpRef* fps,
                      const CandParam* cand, CandRecord* rec, int n_max, const int* n_dev, int n_full);
  // A launch of items: candidate generation, the search kernels, the per-item argmax
  // and, for warm items, the fallback decided and searched on the device.
  prnu_status step(Context& ctx, const Shape& sh, int dtype, const FrameRef* frames, const FpRef* fps,
                   const StepDev& d);
  hipEvent_t prof_event();
  void prof_begin(int k);
  void prof_end(int k, int nc, double bytes);
  void prof_collect();  // after the stream has been synchronised
};

struct ServingEngine;  // serving.hip
struct ServingDeleter {
  void operator()(ServingEngine* e) const;
};

class Context {
 public:
  int device = 0;
  std::mutex mu;     // synchronous calls (one at a time on the synchronous runner)
  std::mutex fp_mu;  // fingerprint table
  std::mutex tw_mu;  // twiddle tables
  std::atomic<bool> failed{false};
  // Host-side fault hook for tests (PRNU_FAULT=launch:N,stage:N): the Nth launch of
  // search kernels, or the Nth frame staging, on this context fails as a device error
  // does, before any of its work is issued.  0 = off.
  int64_t fault_launch = 0, fault_stage = 0;
  std::atomic<int64_t> n_launch{0}, n_stage{0};
  bool inject(int64_t at, std::atomic<int64_t>& count) { return at > 0 && ++count == at; }
  uint64_t hbm_budget = 0;
  int max_slots = 0;
  uint32_t flags = 0;
  std::string tune_cache;
  std::mutex tune_mu;                   // schedule table and tuning
  std::map<ShapeKey, Schedule> schedules;
  uint64_t tune_cap_bytes = 8ull << 30; // workspace limit of a tuning trial

  std::map<int, c32*> tw;
  std::map<prnu_fp, Fingerprint> fps;
  prnu_fp next_fp = 0;

  Runner runner;  // synchronous path
  DevBuf stage_dev, stage_tight, stage_scale, dev_cand, dev_rec, dev_frefs, dev_fprefs, dev_proj;
  // synchronous searches: items, candidate lists, fallback list, chain state, results
  DevBuf dev_items, dev_outs, dev_site, dev_fbc, dev_fbs, dev_fbr, dev_ndev, dev_state, dev_best, dev_res, dev_lists;
  HostBuf host_items, host_outs, host_res, host_lists;
  DevBuf res_ws, res_in, res_out;  // residual extraction: workspace, image and output staging
  HostBuf stage_pinned;             // pinned staging of host frames for the synchronous calls
  HostBuf res_pinned, res_pinned_out;  // residual extraction: pinned input and output staging
  HostBuf host_cand, host_rec, host_refs;

  std::unique_ptr<ServingEngine, ServingDeleter> serving;

  ~Context();
  prnu_status hip_fail(hipError_t e, const char* what);
  const c32* twiddles(int kind, int L);
  // The table if it exists already (never allocates), else null.
  const c32* find_twiddles(int kind, int L);
  // Look up a fingerprint (copy) under fp_mu.
  bool get_fp(prnu_fp h, Fingerprint& out);
  prnu_status stage_frames(const prnu_frames* fr, std::vector<FrameRef>& refs);
  prnu_status evaluate(const Shape& sh, int dtype, const std::vector<CandParam>& params, std::vector<CandRecord>& recs,
                       const std::vector<float>* proj = nullptr);
  // Per-candidate records of the full grid of opts on staged frame `frame`.
  prnu_status score_full(const Shape& sh, int dtype, const prnu_grid& g, int frame, std::vector<CandRecord>& recs);
  prnu_status search(const Fingerprint& fp, const prnu_frames* fr, const prnu_search_opts* o, prnu_frame_result* out);
  prnu_status refine(const Shape& sh, int dtype, int F, const prnu_search_opts* o,
                     const std::vector<std::pair<double, double>>& inits, prnu_frame_result* out);
  prnu_status upload_refs(const std::vector<FrameRef>& frames, const Fingerprint& fp);
  ServingEngine* engine();
  void shutdown_serving();
  // Schedule of a shape, tuned on runner r at first use unless tuning is off.
  prnu_status schedule(const Shape& sh, int dtype, Runner& r, Schedule& out);
  prnu_status tune(const Shape& sh, int dtype, Runner& r, Schedule& out);
  void load_tune_cache();
  void save_tune_cache();
};

// Zero-bordered device copy of n frames (f32 or bf16 bits) from host or device memory.
// Frames into the zero-bordered device layout on stream s.  Host frames go through
// `pinned` when given (pageable caller memory), else straight from their memory.
prnu_status stage_padded(Context& ctx, hipStream_t s, const prnu_frames* fr, DevBuf& tight, DevBuf& padded,
                         HostBuf* pinned = nullptr);

}  // namespace prnu
