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
#include <vector>

#include "../../include/prnu.h"
#include "kernels.hpp"

namespace prnu {

prnu_status fail(prnu_status s, const char* fmt, ...);

struct DevBuf {
  void* ptr = nullptr;
  size_t cap = 0;
  hipError_t reserve(size_t n);
  void release();
};

struct HostBuf {
  void* ptr = nullptr;
  size_t cap = 0;
  hipError_t reserve(size_t n);
  void release();
};

struct Fingerprint {
  int M = 0, N = 0;
  c32* FK = nullptr;  // packed column spectrum of K - mean, [M][N/2]
  double mean = 0.0, norm = 0.0;
};

struct Cand {
  double scale, rot_deg;
};

// Frames staged on the device in the zero-bordered layout (see kernels.hpp).
struct FrameSource {
  const void* data = nullptr;
  int dtype = 0;
  const float* scale = nullptr;
  int radius = 0;
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

struct ServingEngine;  // serving.hip
struct ServingDeleter {
  void operator()(ServingEngine* e) const;
};

double grid_node(int k, int n, double lo, double hi);
double local_node(int k, int n, double centre, double step);
void full_candidates(const prnu_grid& g, std::vector<Cand>& out);
void local_candidates(const prnu_search_opts& o, double cs, double ct, std::vector<Cand>& out);
CandParam make_param(const Cand& c, int frame);
prnu_status check_shape(int M, int N, int radius);
prnu_status validate_opts(const prnu_search_opts* o);
prnu_status validate_frames(const prnu_frames* fr, const Fingerprint& fp);
int argmax_records(const CandRecord* r, int n);
void fill_result(prnu_frame_result& out, const CandRecord& r, const Cand& c, int idx);

struct Context {
  int device = 0;
  hipStream_t stream = nullptr;
  std::mutex mu;  // serialises calls that use the synchronous path's stream and workspace
  bool failed = false;
  uint64_t hbm_budget = 0;
  int max_slots = 0;
  std::string tune_cache;
  int batch_override = 0;
  double batch_bytes = 512.0 * 1024 * 1024;

  std::map<int, c32*> tw;
  std::map<prnu_fp, Fingerprint> fps;
  prnu_fp next_fp = 0;

  DevBuf ws_inter, ws_band, ws_win, ws_norm, ws_energy;
  DevBuf stage_dev, stage_tight, stage_scale, dev_cand, dev_rec;
  HostBuf host_cand, host_rec;

  bool prof_on = false;
  KernelStat prof[PRNU_NUM_KERNELS];
  std::vector<ProfEvent> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;

  std::unique_ptr<ServingEngine, ServingDeleter> serving;

  ~Context();
  prnu_status hip_fail(hipError_t e, const char* what);
  const c32* twiddles(int kind, int L);
  int batch_size(const Shape& sh) const;
  prnu_status ensure_workspace(const Shape& sh, int nc);
  prnu_status run_candidates(const Fingerprint& fp, const FrameSource& src, const CandParam* cand_dev,
                             CandRecord* rec_dev, int n);
  prnu_status stage_frames(const prnu_frames* fr, int radius, FrameSource& src);
  prnu_status evaluate(const Fingerprint& fp, const FrameSource& src, const std::vector<CandParam>& params,
                       std::vector<CandRecord>& recs);
  prnu_status search(const Fingerprint& fp, const prnu_frames* fr, const prnu_search_opts* o, prnu_frame_result* out);
  hipEvent_t prof_event();
  void prof_begin(int k);
  void prof_end(int k, int nc, double bytes);
  void prof_collect();
  void shutdown_serving();
  bool fp_in_use(prnu_fp fp);
};

}  // namespace prnu
