// Device-side candidate generation, per-frame argmax and the warm-start chain
// (launch interface, host side).
//
// A launch of the search kernels carries items: each item is one frame of one video
// with its candidate list (a segment of the launch's list).  Around the search kernels:
//   k_gen        writes every item's candidates (inverse-warp coefficients and the
//                (scale, rotation) pairs) from a grid description: the full grid, a
//                local grid around a centre held on the device, or an explicit list;
//   k_argmax     reduces each item's records to its best candidate (FP64 compare,
//                lowest index on ties, NaN never wins), folds it into the frame's
//                running best and, for a warm frame, decides on the device whether
//                the full grid must follow (local best below the fallback level);
//   k_plan       lays the fallback grids of the items that need one end to end and
//                writes their total, which sizes the device-counted launch set that
//                searches them;
//   k_fill       writes those fallback candidates;
//   k_argmax     (merge phase) folds each fallback segment into its frame's best
//                (earlier candidates win ties) and commits the frame: its result
//                record and the centre of the video's next local grid.
// No host round trip is needed between the frames of a chained video.
#pragma once

#include "../../include/prnu.h"
#include "kernels.hpp"

namespace prnu {

// A candidate's (scale, rotation in degrees), kept beside its coefficients.
struct CandSite {
  double s, t;
};

// Warm-start state of one video: the centre of its next local grid.
struct ChainState {
  double cs, ct;
  int32_t have;  // a centre exists (a previous frame, or the caller's initial transform)
  int32_t pad;
};

// Running best of the frame being searched.
struct FrameBest {
  CandRecord rec;
  double s, t;
  int32_t index;  // in the frame's evaluated list; -1: no finite score yet
  int32_t n_eval;
  int32_t fell_back;
  int32_t pad;
};

enum GenKind { kGenFull = 0, kGenLocal = 1, kGenList = 2 };

// A candidate grid, scale-major: kGenFull is ns x nr uniform nodes over
// [lo0, hi0] x [lo1, hi1]; kGenLocal is ns x nr nodes centre + (k - (n - 1) / 2) step
// around the centre in *centre (steps lo0, lo1); kGenList is list[0 .. n).
struct GridGen {
  int32_t kind;
  int32_t ns, nr;
  int32_t pad;
  double lo0, hi0, lo1, hi1;
  const ChainState* centre;
  const CandSite* list;
};

enum ItemMode {
  kModePlain = 0,   // the frame's only segment: commit
  kModeWarm = 1,    // a local grid: commit, or defer to the full-grid fallback
  kModeRefine = 2,  // one refinement iteration: best of the segment for the host; the
                    // frame's best so far is committed (a later iteration overwrites it)
};

struct ItemDesc {
  GridGen gen;     // the item's candidates
  GridGen full;    // kModeWarm: the fallback grid (kGenFull)
  ChainState* state;            // chained items: the video's state (updated at commit)
  FrameBest* best;              // the frame's running best
  prnu_frame_result* result;    // chained items: where the frame's result is written
  double fallback_pce;
  int32_t n;       // candidates of gen
  int32_t off;     // first candidate in the launch's list
  int32_t slot;    // frame slot in the launch's frame table
  int32_t fslot;   // fingerprint slot in the launch's fingerprint table
  int32_t mode;
  int32_t merge;   // kModeRefine: fold into the running best of earlier iterations
  int32_t fb_n;    // kModeWarm: candidates of the fallback grid
  int32_t iter;    // kModeRefine: the iteration (1-based), reported with the result
};

// Written by the device per item.
struct ItemOut {
  int32_t need;    // kModeWarm: the fallback grid follows
  int32_t fb_off;  // its first candidate in the fallback list
  int32_t seg_index;  // kModeRefine: best candidate of the segment (-1: none)
  int32_t pad;
  double seg_s, seg_t, seg_pce;
};

// Device helpers of the launches above (chain.hip).  items/outs: device arrays of n
// items; cand/site: the launch's candidate list; rec its records; fb_* the fallback
// list (max_fb entries) and n_dev its device-written length.
hipError_t launch_gen(const ItemDesc* items, int n, int max_n, CandParam* cand, CandSite* site, hipStream_t s);
hipError_t launch_argmax(const ItemDesc* items, int n, ItemOut* outs, const CandRecord* rec, const CandSite* site,
                         bool merge_fallback, const CandRecord* fb_rec, const CandSite* fb_site, hipStream_t s);
hipError_t launch_plan(const ItemDesc* items, int n, ItemOut* outs, int* n_dev, hipStream_t s);
hipError_t launch_fill(const ItemDesc* items, int n, const ItemOut* outs, const int* n_dev, int max_fb,
                       CandParam* fb_cand, CandSite* fb_site, hipStream_t s);
// Device state of a chained video before its first frame: the caller's initial
// transform, or no centre (a warm item whose video has no centre yet is searched on its
// full grid alone, like a first frame).
hipError_t launch_chain_init(ChainState* st, int has_init, double cs, double ct, hipStream_t s);
// Up to kBlobBytes bytes written to device memory dst by a kernel that takes them as
// its argument (no host-to-device copy, so nothing reads host memory later).
constexpr int kBlobBytes = 1024;
struct Blob {
  unsigned char b[kBlobBytes];
  int32_t n;
};
hipError_t launch_put(const Blob& blob, void* dst, hipStream_t s);
// Records of candidates [0, n) to four device arrays (any may be null).
hipError_t launch_scatter(const CandRecord* rec, int n, double* pce, double* rho, int32_t* dx, int32_t* dy,
                          hipStream_t s);

}  // namespace prnu
