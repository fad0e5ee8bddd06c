// Host runtime of libdfr: tile choice and the tuned-shape cache, launch
// geometry, per-(device, stream) workspaces and the graph-replayed batch.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "launch.hpp"

namespace dfr {

constexpr int kLdsMaxFloats = 16384;  // 64 KiB of LDS per work-group for staged source

// Tile for a reprojection: `requested` if nonzero, else the tuned cache
// entry for this kind of map, else a heuristic that fits the LDS budget.
// pref: the untuned shape to try first (0: the forward's default for the
// interpolation).
int choose_tile(const FramePlan &P, int32_t out_h, int32_t out_w, int interp, int requested,
                bool batch, int lds_factor = 1, int pref = 0);

// Key under which tuned tiles are cached: kind, interpolation, SIP order and
// coarse classes of the map's magnification and rotation.
std::string tune_key(const FramePlan &P, int32_t out_h, int32_t out_w, int interp, bool batch);
void tune_store(const std::string &key, int tile);
// Cached tile for `key`, 0 if none (caller holds tune_mutex_for_batch()).
int tuned_tile(const std::string &key);
std::mutex &tune_mutex_for_batch();

// Host set-up of a single-image FP32 call (the FP64 plan, the tile choice
// and the launch geometry), cached per geometry: the key holds the bytes of
// both WCS and their SIP coefficients, the shapes, the interpolation, the
// requested tile and the tuned-tile cache's generation, so a hit is exactly
// what the set-up would compute again.  Image pointers and the per-call
// options (cubic a, NaN outside, debug output) are filled in on every call.
// The backward's set-up passes lds_factor (copies of the box it keeps), its
// untuned tile preference, and two_rows (4-row tiles run as their 2-row
// sibling of the same width).
void single_setup(const float *src, int32_t src_h, int32_t src_w, int64_t src_pitch,
                  const dfr_wcs &sw, const dfr_wcs &tw, int32_t out_h, int32_t out_w,
                  float *out, float *footprint, int interp, const dfr_options &o, FramePlan &P,
                  TileGeom &G, TileShape &ts, int lds_factor = 1, int pref = 0,
                  bool two_rows = false);

// lds_factor: copies of the source box a kernel keeps (backward: 2).
void make_geom(const FramePlan &P, int32_t out_h, int32_t out_w, int interp, int tile,
               const dfr_options &o, TileGeom &G, TileShape &ts, int lds_factor = 1);

// Scratch owned by the library for one (device, stream): device memory for
// partial sums, the batch frame table and its counter, pinned staging for
// the frame table, and the instantiated batch graphs.  Work on one stream is
// ordered, so reusing the buffers call after call is safe; every function
// here must be called with workspace_mutex() held.
struct BatchGraph {
  TileGeom geom;
  int n, interp, np, sord, grid, models;
  void *plans_dev;
  void *plans_host;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

struct Workspace {
  int device = -1;
  hipStream_t stream = nullptr;
  void *buf = nullptr;  // device scratch
  size_t cap = 0;
  FramePlan *host_plans = nullptr;  // pinned staging of the batch frame table
  size_t host_cap = 0;              // in frames
  hipEvent_t staged = nullptr;      // recorded after the last batch that read host_plans
  bool staged_pending = false;
  std::vector<BatchGraph> graphs;
  int *ctl = nullptr;      // backward control words: max|g| bits in two alternating slots
  int ctl_slot = 0;        // the slot the next backward call uses (zero)
  bool ctl_dirty = true;   // ctl may be non-zero (new, or a call stopped part-way)
};

std::mutex &workspace_mutex();
Workspace *workspace(hipStream_t stream);
// Device scratch of at least `bytes` for the workspace, into *buf:
// DFR_E_DEVICE if waiting for the stream's earlier work (before replacing a
// smaller buffer) fails, DFR_E_NOMEM if the allocation fails.
dfr_status workspace_buffer(Workspace *w, size_t bytes, void **buf);
// The workspace's backward control words (allocated on first use): slot
// ctl_slot is zero when the next kernel on its stream runs (each call's
// first kernel zeroes the other slot, which the next call uses); a call
// that stops part-way marks them dirty, and they are zeroed here, by a
// kernel.
dfr_status workspace_control(Workspace *w, int **ctl);
void release_workspaces();

// What a batch run produces besides the default per-frame outputs.
struct BatchRun {
  const CoaddOut *coadd = nullptr;  // stack the frames into these sums
  int64_t crop_items = -1;          // >= 0: per-frame windows, this many work items
  int32_t *reach_host = nullptr;    // only the model prepass: its reach boxes, 4 per frame
};

// Reproject a batch in one persistent launch; `graph` replays a cached HIP
// graph (frame-table copy, per-cell models of every frame when `models`,
// counter reset, persistent kernel).  The coadd, cropped and reach-only
// runs launch eagerly (their output pointers are kernel arguments, or the
// host waits).
dfr_status run_batch(const std::vector<FramePlan> &plans, const TileGeom &G, int interp, int np,
                     int max_sord, bool models, hipStream_t stream, bool graph,
                     const BatchRun &run = BatchRun());

}  // namespace dfr
