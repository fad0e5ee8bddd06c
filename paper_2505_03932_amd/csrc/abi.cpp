// extern "C" entry points of libdfr (declared in include/dfr.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "cell_model.hpp"
#include "dfr.h"
#include "launch.hpp"
#include "plan.hpp"
#include "runtime.hpp"
#include "scratch.hpp"

static_assert(dfr::kScratchBytes == DFR_NOALLOC_SCRATCH_BYTES, "scratch size in the header");

using namespace dfr;

namespace {

dfr_status resolve_options(const dfr_options *opt, dfr_options &o) {
  dfr_options_init(&o);
  if (!opt) return DFR_OK;
  if (opt->size != sizeof(dfr_options)) return DFR_E_ARG;
  o = *opt;
  if (o.precision < DFR_PREC_F32 || o.precision > DFR_PREC_F32_ANCHOR) return DFR_E_UNSUPPORTED;
  if (!std::isfinite(o.cubic_a)) return DFR_E_ARG;
  if (o.tile < 0 || o.tile > kTileCount) return DFR_E_ARG;
  if (o.reserved_ != 0) return DFR_E_ARG;
  return DFR_OK;
}

bool is_f32(const dfr_options &o) {
  return o.precision == DFR_PREC_F32 || o.precision == DFR_PREC_F32_ANCHOR;
}

// FP32 forward of one frame with tile `tile`: the per-cell position models
// first where the map allows them (default precision, target without SIP;
// the table lives in the stream's workspace, so the caller holds
// workspace_mutex() from here until every launch reading it is queued).
dfr_status models_for(FramePlan &P, int32_t out_h, int32_t out_w, const dfr_options &o,
                      hipStream_t st) {
  P.models = nullptr;
  if (o.precision != DFR_PREC_F32 || P.t_order > 0) return DFR_OK;
  const int ncx = (out_w + kCell - 1) / kCell, ncy = (out_h + kCell - 1) / kCell;
  void *buf = nullptr;
  dfr_status s = workspace_buffer(workspace(st), (size_t)ncx * ncy * sizeof(CellModel), &buf);
  if (s != DFR_OK) return s;
  CellModel *table = static_cast<CellModel *>(buf);
  P.models = table;
  return launch_cell_models(P, ncx, ncy, table, st) == hipSuccess ? DFR_OK : DFR_E_DEVICE;
}

bool interp_ok(int interp) {
  return interp == DFR_NEAREST || interp == DFR_BILINEAR || interp == DFR_BICUBIC;
}

// Argument checks shared by the single-image entry points.
dfr_status check_single(const float *src, int32_t src_h, int32_t src_w, int64_t src_pitch,
                        const dfr_wcs *src_wcs, const dfr_wcs *tgt_wcs, int32_t out_h,
                        int32_t out_w, int interp) {
  if (!src_wcs || !tgt_wcs) return DFR_E_NULL;
  if (src_h < 0 || src_w < 0 || out_h < 0 || out_w < 0) return DFR_E_SHAPE;
  if (src_h > 0 && src_w > 0) {
    if (!src) return DFR_E_NULL;
    if (src_pitch < src_w) return DFR_E_SHAPE;
  }
  dfr_status s;
  if ((s = check_wcs(src_wcs, true)) != DFR_OK) return s;
  if ((s = check_wcs(tgt_wcs, false)) != DFR_OK) return s;
  if (!interp_ok(interp)) return DFR_E_UNSUPPORTED;
  return DFR_OK;
}

// Batch tune key: the interpolation, the padded SIP order, the frame count
// and the output size class (frames of a stack differ in rotation and scale).
std::string batch_key(const std::vector<FramePlan> &plans, int32_t out_h, int32_t out_w,
                      int interp, int max_sord) {
  char key[128];
  int mb = (int)std::lround(std::log2(std::max(1.0, (double)out_h * out_w)));
  std::snprintf(key, sizeof(key), "batch:i%d:s%d:n%d:o%d", interp, std::min(max_sord, 6),
                (int)plans.size(), mb);
  return key;
}

// Geometry for a batch with tile `t`: the LDS budget covers the largest
// estimated source box over the frames.
void batch_geom(const std::vector<FramePlan> &plans, int32_t out_h, int32_t out_w, int interp,
                int t, const dfr_options &o, TileGeom &G, int &np) {
  TileShape ts;
  make_geom(plans[0], out_h, out_w, interp, t, o, G, ts);
  int64_t need = 0;
  for (auto &P : plans) need = std::max<int64_t>(need, estimate_lds_floats(P, out_h, out_w, ts, interp));
  G.lds_cap = need <= kLdsMaxFloats ? (int32_t)need : 0;
  np = ts.np;
}

dfr_status prepare_batch(int32_t n, const dfr_frame *frames, const dfr_wcs *tgt_wcs,
                         int32_t out_h, int32_t out_w, int interp, float *const *outs,
                         float *const *footprints, const dfr_options *opt,
                         std::vector<FramePlan> &plans, TileGeom &G, int &tile, int &np,
                         int &max_sord, bool stack = false) {
  // stack: a coadd, whose frames have no outputs of their own (outs unused)
  if (n < 0) return DFR_E_ARG;
  if (n > 0 && (!frames || (!outs && !stack))) return DFR_E_NULL;
  if (!tgt_wcs) return DFR_E_NULL;
  if (out_h < 0 || out_w < 0) return DFR_E_SHAPE;
  if (!interp_ok(interp)) return DFR_E_UNSUPPORTED;
  dfr_status s;
  if ((s = check_wcs(tgt_wcs, false)) != DFR_OK) return s;
  dfr_options o;
  if ((s = resolve_options(opt, o)) != DFR_OK) return s;
  if (!is_f32(o)) return DFR_E_UNSUPPORTED;
  if (o.debug_positions) return DFR_E_ARG;
  if ((int64_t)n * (((int64_t)out_h * out_w + 1023) / 1024) > 0x7fffffffLL) return DFR_E_SHAPE;
  for (int i = 0; i < n; ++i) {
    const dfr_frame &f = frames[i];
    if (f.h < 0 || f.w < 0) return DFR_E_SHAPE;
    if (f.h > 0 && f.w > 0) {
      if (!f.src) return DFR_E_NULL;
      if (f.pitch < f.w) return DFR_E_SHAPE;
    }
    if ((s = check_wcs(&f.wcs, true)) != DFR_OK) return s;
    if (!stack && (int64_t)out_h * out_w > 0 && !outs[i]) return DFR_E_NULL;
  }
  plans.clear();
  if (n == 0 || out_h == 0 || out_w == 0) {
    std::memset(&G, 0, sizeof(G));
    return DFR_OK;
  }
  plans.resize(n);
  max_sord = 0;
  for (int i = 0; i < n; ++i) {
    const dfr_frame &f = frames[i];
    const float *src = (f.h > 0 && f.w > 0) ? f.src : nullptr;
    build_plan(src, f.h, f.w, f.pitch, f.wcs, *tgt_wcs, out_h, out_w, stack ? nullptr : outs[i],
               (footprints && !stack) ? footprints[i] : nullptr, plans[i]);
    max_sord = std::max(max_sord, plans[i].s_order);
  }
  // run-time-order kernel for high orders and whenever the target has SIP
  if (max_sord > 5 || plans[0].t_order > 0) max_sord = 6;
  tile = o.tile;
  if (tile == 0 && !stack) {
    std::lock_guard<std::mutex> lk(tune_mutex_for_batch());
    tile = tuned_tile(batch_key(plans, out_h, out_w, interp, max_sord));
  }
  if (tile == 0) tile = stack ? kCoaddTile : choose_tile(plans[0], out_h, out_w, interp, 0, true);
  batch_geom(plans, out_h, out_w, interp, tile, o, G, np);
  return DFR_OK;
}

// Time every tile shape (two warm launches, then the best of three timed
// ones) and return the fastest in `best`.
template <typename Run>
dfr_status time_candidates(Run &run, hipStream_t st, int &best) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return DFR_E_DEVICE;
  float best_ms = 1e30f;
  best = kDefaultTile;
  dfr_status status = DFR_OK;
  for (int t = 1; t <= kTileCount && status == DFR_OK; ++t) {
    float ms_min = 1e30f;
    for (int rep = 0; rep < 5; ++rep) {
      float ms = 0.0f;
      if (hipEventRecord(e0, st) != hipSuccess || !run(t) || hipEventRecord(e1, st) != hipSuccess ||
          hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        status = DFR_E_DEVICE;
        break;
      }
      if (rep >= 2) ms_min = std::min(ms_min, ms);
    }
    if (ms_min < best_ms) {
      best_ms = ms_min;
      best = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return status;
}

}  // namespace

// A reprojection geometry prepared once for many images (dfr_plan_*): the
// frame plan without its image pointers, the tile geometry, and the per-cell
// models in device memory the plan owns.
struct dfr_plan {
  dfr::FramePlan P;
  dfr::TileGeom G;
  int interp = 0, np = 1, device = 0;
  dfr::CellModel *models = nullptr;
};

extern "C" {

void dfr_options_init(dfr_options *opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->size = sizeof(dfr_options);
  opt->precision = DFR_PREC_F32;
  opt->cubic_a = -0.5;
  opt->nan_outside = 0;
  opt->tile = 0;
  opt->debug_positions = nullptr;
  opt->deterministic = 0;
  opt->reserved_ = 0;
}

dfr_status dfr_reproject(const float *src, int32_t src_h, int32_t src_w, int64_t src_pitch,
                         const dfr_wcs *src_wcs, const dfr_wcs *tgt_wcs, int32_t out_h,
                         int32_t out_w, dfr_interp interp, float *out, float *footprint,
                         const dfr_options *opt, void *stream) {
  dfr_status s = check_single(src, src_h, src_w, src_pitch, src_wcs, tgt_wcs, out_h, out_w,
                              (int)interp);
  if (s != DFR_OK) return s;
  dfr_options o;
  if ((s = resolve_options(opt, o)) != DFR_OK) return s;
  if (out_h == 0 || out_w == 0) return DFR_OK;
  if (!out) return DFR_E_NULL;
  if (src_h == 0 || src_w == 0) src = nullptr;
  FramePlan P;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipError_t e;
  if (is_f32(o)) {
    TileGeom G;
    TileShape ts;
    single_setup(src, src_h, src_w, src_pitch, *src_wcs, *tgt_wcs, out_h, out_w, out, footprint,
                 (int)interp, o, P, G, ts);
    std::lock_guard<std::mutex> lk(workspace_mutex());
    if ((s = models_for(P, out_h, out_w, o, st)) != DFR_OK) return s;
    e = launch_forward_f32(P, G, (int)interp, ts.np, st);
  } else {
    build_plan(src, src_h, src_w, src_pitch, *src_wcs, *tgt_wcs, out_h, out_w, out, footprint, P);
    TrigPlan T;
    build_trig_plan(*src_wcs, *tgt_wcs, T);
    TileGeom G;
    TileShape ts;
    make_geom(P, out_h, out_w, (int)interp, kDefaultTile, o, G, ts);
    e = launch_forward_f64(P, T, G, (int)interp, o.precision == DFR_PREC_TRIG_F64, st);
  }
  return e == hipSuccess ? DFR_OK : DFR_E_DEVICE;
}

dfr_status dfr_reproject_noalloc(const float *src, int32_t src_h, int32_t src_w,
                                 int64_t src_pitch, const dfr_wcs *src_wcs,
                                 const dfr_wcs *tgt_wcs, int32_t out_h, int32_t out_w,
                                 dfr_interp interp, float *out, float *footprint,
                                 const dfr_options *opt, void *stream) {
  dfr_status s = check_single(src, src_h, src_w, src_pitch, src_wcs, tgt_wcs, out_h, out_w,
                              (int)interp);
  if (s != DFR_OK) return s;
  dfr_options o;
  if ((s = resolve_options(opt, o)) != DFR_OK) return s;
  if (out_h == 0 || out_w == 0) return DFR_OK;
  if (!out) return DFR_E_NULL;
  if (src_h == 0 || src_w == 0) src = nullptr;
  FramePlan P;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipError_t e;
  if (is_f32(o)) {
    TileGeom G;
    TileShape ts;
    single_setup(src, src_h, src_w, src_pitch, *src_wcs, *tgt_wcs, out_h, out_w, out, footprint,
                 (int)interp, o, P, G, ts);
    P.models = nullptr;
    if (o.precision == DFR_PREC_F32 && P.t_order == 0) {
      // the model table goes to the device's fixed scratch, not the
      // stream's workspace: refuse a grid whose table does not fit before
      // any device call
      const int64_t ncx = (out_w + kCell - 1) / kCell, ncy = (out_h + kCell - 1) / kCell;
      if (ncx * ncy * (int64_t)sizeof(CellModel) > (int64_t)kScratchBytes) return DFR_E_LIMIT;
      void *table = nullptr;
      if (scratch_address(&table) != hipSuccess) return DFR_E_DEVICE;
      CellModel *models = static_cast<CellModel *>(table);
      P.models = models;
      if (launch_cell_models(P, (int)ncx, (int)ncy, models, st) != hipSuccess)
        return DFR_E_DEVICE;
    }
    e = launch_forward_f32(P, G, (int)interp, ts.np, st);
  } else {
    build_plan(src, src_h, src_w, src_pitch, *src_wcs, *tgt_wcs, out_h, out_w, out, footprint, P);
    TrigPlan T;
    build_trig_plan(*src_wcs, *tgt_wcs, T);
    TileGeom G;
    TileShape ts;
    make_geom(P, out_h, out_w, (int)interp, kDefaultTile, o, G, ts);
    e = launch_forward_f64(P, T, G, (int)interp, o.precision == DFR_PREC_TRIG_F64, st);
  }
  return e == hipSuccess ? DFR_OK : DFR_E_DEVICE;
}

dfr_status dfr_reproject_batch(int32_t n, const dfr_frame *frames, const dfr_wcs *tgt_wcs,
                               int32_t out_h, int32_t out_w, dfr_interp interp,
                               float *const *outs, float *const *footprints,
                               const dfr_options *opt, void *stream) {
  std::vector<FramePlan> plans;
  int tile = 0, np = 0, max_sord = 0;
  TileGeom G;
  dfr_status s = prepare_batch(n, frames, tgt_wcs, out_h, out_w, (int)interp, outs, footprints,
                               opt, plans, G, tile, np, max_sord);
  if (s != DFR_OK || plans.empty() || G.n_tiles == 0) return s;
  dfr_options o;
  resolve_options(opt, o);
  return run_batch(plans, G, (int)interp, np, max_sord, o.precision == DFR_PREC_F32,
                   reinterpret_cast<hipStream_t>(stream), true);
}

dfr_status dfr_coadd_batch(int32_t n, const dfr_frame *frames, const dfr_wcs *tgt_wcs,
                           int32_t out_h, int32_t out_w, dfr_interp interp, float *sum_wf,
                           float *sum_f, float *coadd, int32_t accumulate,
                           const dfr_options *opt, void *stream) {
  std::vector<FramePlan> plans;
  int tile = 0, np = 0, max_sord = 0;
  TileGeom G;
  dfr_status s = prepare_batch(n, frames, tgt_wcs, out_h, out_w, (int)interp, nullptr, nullptr,
                               opt, plans, G, tile, np, max_sord, true);
  if (s != DFR_OK) return s;
  if (out_h == 0 || out_w == 0) return DFR_OK;
  if (!sum_wf || !sum_f) return DFR_E_NULL;
  dfr_options o;
  resolve_options(opt, o);
  const CoaddOut C{sum_wf, sum_f, coadd, accumulate ? 1 : 0};
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (plans.empty()) {
    // an empty stack: the sums stay (accumulate) or become 0
    FramePlan P;
    build_plan(nullptr, 0, 0, 0, *tgt_wcs, *tgt_wcs, out_h, out_w, nullptr, nullptr, P);
    TileShape ts;
    make_geom(P, out_h, out_w, (int)interp, o.tile ? o.tile : kCoaddTile, o, G, ts);
    G.lds_cap = 0;
    return launch_coadd_f32(nullptr, 0, 0, G, (int)interp, ts.np, C, st) == hipSuccess
               ? DFR_OK
               : DFR_E_DEVICE;
  }
  BatchRun run;
  run.coadd = &C;
  return run_batch(plans, G, (int)interp, np, max_sord, o.precision == DFR_PREC_F32, st, false,
                   run);
}

dfr_status dfr_batch_boxes(int32_t n, const dfr_frame *frames, const dfr_wcs *tgt_wcs,
                           int32_t out_h, int32_t out_w, dfr_interp interp,
                           const dfr_options *opt, void *stream, int32_t *boxes) {
  if (n > 0 && !boxes) return DFR_E_NULL;
  std::vector<FramePlan> plans;
  int tile = 0, np = 0, max_sord = 0;
  TileGeom G;
  dfr_status s = prepare_batch(n, frames, tgt_wcs, out_h, out_w, (int)interp, nullptr, nullptr,
                               opt, plans, G, tile, np, max_sord, true);
  if (s != DFR_OK) return s;
  if (plans.empty() || G.n_tiles == 0) {
    for (int i = 0; i < 4 * n; ++i) boxes[i] = 0;
    return DFR_OK;
  }
  dfr_options o;
  resolve_options(opt, o);
  std::vector<int32_t> reach(4 * (size_t)n);
  BatchRun run;
  run.reach_host = reach.data();
  if ((s = run_batch(plans, G, (int)interp, np, max_sord, o.precision == DFR_PREC_F32,
                     reinterpret_cast<hipStream_t>(stream), false, run)) != DFR_OK)
    return s;
  for (int i = 0; i < n; ++i) {
    const int32_t *r = &reach[4 * (size_t)i];
    int32_t *b = boxes + 4 * (size_t)i;
    if (r[0] == -1) {  // no model table: the whole grid
      b[0] = b[1] = 0;
      b[2] = out_w;
      b[3] = out_h;
    } else if (r[1] == 0) {  // no cell reaches the source
      b[0] = b[1] = b[2] = b[3] = 0;
    } else {
      const int64_t x0 = (int64_t)(kReachBig - r[0]) * kCell, y0 = (int64_t)(kReachBig - r[2]) * kCell;
      const int64_t x1 = std::min<int64_t>((int64_t)r[1] * kCell, out_w);
      const int64_t y1 = std::min<int64_t>((int64_t)r[3] * kCell, out_h);
      b[0] = (int32_t)x0;
      b[1] = (int32_t)y0;
      b[2] = (int32_t)std::max<int64_t>(x1 - x0, 0);
      b[3] = (int32_t)std::max<int64_t>(y1 - y0, 0);
    }
  }
  return DFR_OK;
}

dfr_status dfr_reproject_batch_cropped(int32_t n, const dfr_frame *frames,
                                       const dfr_wcs *tgt_wcs, int32_t out_h, int32_t out_w,
                                       dfr_interp interp, const int32_t *boxes,
                                       float *const *outs, float *const *footprints,
                                       const dfr_options *opt, void *stream) {
  if (n > 0 && (!boxes || !outs)) return DFR_E_NULL;
  for (int i = 0; i < n; ++i) {
    const int32_t *b = boxes + 4 * (size_t)i;
    if (b[0] < 0 || b[1] < 0 || b[2] < 0 || b[3] < 0 || (int64_t)b[0] + b[2] > out_w ||
        (int64_t)b[1] + b[3] > out_h)
      return DFR_E_SHAPE;
    if ((int64_t)b[2] * b[3] > 0 && !outs[i]) return DFR_E_NULL;
  }
  std::vector<FramePlan> plans;
  int tile = 0, np = 0, max_sord = 0;
  TileGeom G;
  dfr_status s = prepare_batch(n, frames, tgt_wcs, out_h, out_w, (int)interp, nullptr, nullptr,
                               opt, plans, G, tile, np, max_sord, true);
  if (s != DFR_OK || plans.empty() || G.n_tiles == 0) return s;
  // each frame's window and the range of global tiles that meet it
  TileShape ts;
  tile_shape(tile, ts);
  int64_t items = 0;
  for (int i = 0; i < n; ++i) {
    const int32_t *b = boxes + 4 * (size_t)i;
    FramePlan &P = plans[i];
    P.out = outs[i];
    P.fp = footprints ? footprints[i] : nullptr;
    P.crop[0] = b[0];
    P.crop[1] = b[1];
    P.crop[2] = b[2];
    P.crop[3] = b[3];
    P.item0 = (int32_t)items;
    P.tile0[0] = b[0] / ts.width;
    P.tile0[1] = b[1] / ts.height;
    P.ntx = 1;
    if ((int64_t)b[2] * b[3] == 0) continue;
    const int tx1 = (b[0] + b[2] - 1) / ts.width, ty1 = (b[1] + b[3] - 1) / ts.height;
    P.ntx = tx1 - P.tile0[0] + 1;
    items += (int64_t)P.ntx * (ty1 - P.tile0[1] + 1);
    if (items > 0x7fffffffLL) return DFR_E_SHAPE;
  }
  dfr_options o;
  resolve_options(opt, o);
  BatchRun run;
  run.crop_items = items;
  return run_batch(plans, G, (int)interp, np, max_sord, o.precision == DFR_PREC_F32,
                   reinterpret_cast<hipStream_t>(stream), false, run);
}

dfr_status dfr_plan_create(int32_t src_h, int32_t src_w, const dfr_wcs *src_wcs,
                           const dfr_wcs *tgt_wcs, int32_t out_h, int32_t out_w,
                           dfr_interp interp, const dfr_options *opt, void *stream,
                           dfr_plan **plan) {
  if (!plan) return DFR_E_NULL;
  *plan = nullptr;
  if (!src_wcs || !tgt_wcs) return DFR_E_NULL;
  if (src_h < 0 || src_w < 0 || out_h < 0 || out_w < 0) return DFR_E_SHAPE;
  dfr_status s;
  if ((s = check_wcs(src_wcs, true)) != DFR_OK) return s;
  if ((s = check_wcs(tgt_wcs, false)) != DFR_OK) return s;
  if (!interp_ok((int)interp)) return DFR_E_UNSUPPORTED;
  dfr_options o;
  if ((s = resolve_options(opt, o)) != DFR_OK) return s;
  if (!is_f32(o)) return DFR_E_UNSUPPORTED;
  if (o.debug_positions) return DFR_E_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DFR_E_DEVICE;
  dfr_plan *pl = new (std::nothrow) dfr_plan();
  if (!pl) return DFR_E_NOMEM;
  pl->device = dev;
  pl->interp = (int)interp;
  build_plan(nullptr, src_h, src_w, src_w, *src_wcs, *tgt_wcs, out_h, out_w, nullptr, nullptr,
             pl->P);
  TileShape ts;
  const int tile = choose_tile(pl->P, out_h, out_w, (int)interp, o.tile, false);
  make_geom(pl->P, out_h, out_w, (int)interp, tile, o, pl->G, ts);
  pl->np = ts.np;
  if (o.precision == DFR_PREC_F32 && pl->P.t_order == 0 && out_h > 0 && out_w > 0) {
    const int ncx = (out_w + kCell - 1) / kCell, ncy = (out_h + kCell - 1) / kCell;
    if (hipMalloc(&pl->models, (size_t)ncx * ncy * sizeof(CellModel)) != hipSuccess) {
      pl->models = nullptr;
      delete pl;
      return DFR_E_NOMEM;
    }
    pl->P.models = pl->models;
    if (launch_cell_models(pl->P, ncx, ncy, pl->models, reinterpret_cast<hipStream_t>(stream)) !=
        hipSuccess) {
      (void)hipFree(pl->models);
      delete pl;
      return DFR_E_DEVICE;
    }
  }
  *plan = pl;
  return DFR_OK;
}

dfr_status dfr_plan_execute(const dfr_plan *plan, const float *src, int64_t src_pitch, float *out,
                            float *footprint, void *stream) {
  if (!plan) return DFR_E_NULL;
  const int32_t h = plan->P.src_h, w = plan->P.src_w;
  if (h > 0 && w > 0) {
    if (!src) return DFR_E_NULL;
    if (src_pitch < w) return DFR_E_SHAPE;
  }
  if (plan->G.out_h == 0 || plan->G.out_w == 0) return DFR_OK;
  if (!out) return DFR_E_NULL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return DFR_E_DEVICE;
  if (dev != plan->device) return DFR_E_ARG;
  FramePlan P = plan->P;
  P.src = (h > 0 && w > 0) ? src : nullptr;
  P.pitch = src_pitch;
  P.out = out;
  P.fp = footprint;
  return launch_forward_f32(P, plan->G, plan->interp, plan->np,
                            reinterpret_cast<hipStream_t>(stream)) == hipSuccess
             ? DFR_OK
             : DFR_E_DEVICE;
}

dfr_status dfr_plan_destroy(dfr_plan *plan) {
  if (!plan) return DFR_OK;
  dfr_status s = DFR_OK;
  if (plan->models && hipFree(plan->models) != hipSuccess) s = DFR_E_DEVICE;
  delete plan;
  return s;
}

dfr_status dfr_reproject_backward(const float *src, int32_t src_h, int32_t src_w,
                                  int64_t src_pitch, const dfr_wcs *src_wcs,
                                  const dfr_wcs *tgt_wcs, int32_t out_h, int32_t out_w,
                                  dfr_interp interp, const float *grad_out, float *grad_src,
                                  double *grad_wcs, const dfr_options *opt, void *stream) {
  dfr_status s = check_single(src, src_h, src_w, src_pitch, src_wcs, tgt_wcs, out_h, out_w,
                              (int)interp);
  if (s != DFR_OK) return s;
  dfr_options o;
  if ((s = resolve_options(opt, o)) != DFR_OK) return s;
  if (!is_f32(o)) return DFR_E_UNSUPPORTED;
  if (std::max(src_wcs->ap_order, src_wcs->bp_order) > 5) return DFR_E_UNSUPPORTED;
  if ((int64_t)out_h * out_w > 0 && !grad_out) return DFR_E_NULL;
  if (src_h == 0 || src_w == 0) src = nullptr;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // the source adjoint is summed in integers in a workspace buffer and
  // converted into grad_src (every entry written)
  const bool det = grad_src && src_h > 0 && src_w > 0;
  FramePlan P;
  o.debug_positions = nullptr;
  TileGeom G;
  TileShape ts;
  // LDS: the source box and, for the source adjoint, its 64-bit integer
  // accumulation copy; 4-row tiles run as their 2-row sibling
  single_setup(src, src_h, src_w, src_pitch, *src_wcs, *tgt_wcs, out_h, out_w, nullptr, nullptr,
               (int)interp, o, P, G, ts, det ? 3 : 1,
               backward_default_tile((int)interp, grad_src != nullptr), true);
  const int ns = backward_sums(P.s_order);
  WcsJacobian J;
  h_jacobian(*src_wcs, *tgt_wcs, J.dh);
  FinishArgs A;
  A.ns = ns;
  A.nr = grad_wcs ? ns - 10 : 0;
  A.J = J;
  A.S = P.s_scale;
  A.grad_wcs = grad_wcs;
  if (grad_wcs) {
    // where each SIP column's total goes in the square AP/BP layouts, and
    // which entries lie above their polynomial's order (zero)
    const int NC = (P.s_order + 1) * (P.s_order + 2) / 2;
    for (int k = 0; k < 2 * NC; ++k) A.col_entry[k] = -1;
    A.n_above = 0;
    int base = 8;
    for (int poly = 0; poly < 2; ++poly) {
      const int o = poly == 0 ? src_wcs->ap_order : src_wcs->bp_order;
      if (o <= 0) continue;
      for (int p = 0; p <= o; ++p)
        for (int q = 0; q <= o; ++q) {
          const int e = base + p * (o + 1) + q;
          if (p + q <= o) {
            const int k = poly * NC + tri_n(P.s_order, p, q);
            A.col_entry[k] = e;
            A.col_deg[k] = p + q;
          } else {
            A.above[A.n_above++] = e;
          }
        }
      base += (o + 1) * (o + 1);
    }
  }
  std::lock_guard<std::mutex> lk(workspace_mutex());
  Workspace *w = workspace(st);
  // workspace: per-tile FP64 partials; for the source adjoint also the
  // 64-bit integer sums; max|g| (as float bits) alternates between two of
  // the workspace's control words
  const size_t pbytes = (size_t)std::max(G.n_tiles, 1) * ns * sizeof(double);
  const size_t qofs = (pbytes + 255) & ~(size_t)255;
  const size_t bytes = det ? qofs + (size_t)src_h * src_w * sizeof(uint64_t) : pbytes;
  void *buf = nullptr;
  int *ctl = nullptr;
  if ((s = workspace_buffer(w, bytes, &buf)) != DFR_OK) return s;
  if ((s = workspace_control(w, &ctl)) != DFR_OK) return s;
  double *part = static_cast<double *>(buf);
  unsigned long long *qacc =
      det ? reinterpret_cast<unsigned long long *>(static_cast<char *>(buf) + qofs) : nullptr;
  int *gmax = ctl + w->ctl_slot, *gmax_next = ctl + (w->ctl_slot ^ 1);
  A.partials = part;
  A.n_blocks = G.n_tiles;
  A.q = qacc;
  A.h = det ? src_h : 0;
  A.w = det ? src_w : 0;
  A.gsrc = grad_src;
  A.gpitch = src_w;
  A.gmax = gmax;
  // zero the integer sums and take max|g| (one kernel), the backward, then
  // grad_src and the WCS gradient (one kernel); a launch that fails leaves
  // the control words dirty
  const bool ok =
      (!det || launch_det_prepare(grad_out, (int64_t)out_h * out_w, qacc,
                                  (int64_t)src_h * src_w, gmax, gmax_next, st) == hipSuccess) &&
      (G.n_tiles <= 0 ||
       launch_backward(P, G, (int)interp, ts.np, grad_out, part, qacc, gmax, st) == hipSuccess) &&
      launch_backward_finish(A, st) == hipSuccess;
  if (!ok) {
    w->ctl_dirty = true;
    return DFR_E_DEVICE;
  }
  if (det) w->ctl_slot ^= 1;
  return DFR_OK;
}

dfr_status dfr_sq_residual(const float *out, const float *ref, const float *mask, int64_t n,
                           double *loss, float *grad_out, void *stream) {
  if (n < 0) return DFR_E_SHAPE;
  if (!loss || (n > 0 && (!out || !ref))) return DFR_E_NULL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256));
  std::lock_guard<std::mutex> lk(workspace_mutex());
  void *buf = nullptr;
  dfr_status s = workspace_buffer(workspace(st), blocks * sizeof(double), &buf);
  if (s != DFR_OK) return s;
  double *part = static_cast<double *>(buf);
  return launch_sq_residual(out, ref, mask, n, part, blocks, loss, grad_out, st) == hipSuccess
             ? DFR_OK
             : DFR_E_DEVICE;
}

dfr_status dfr_autotune(const float *src, int32_t src_h, int32_t src_w, int64_t src_pitch,
                        const dfr_wcs *src_wcs, const dfr_wcs *tgt_wcs, int32_t out_h,
                        int32_t out_w, dfr_interp interp, float *out, float *footprint,
                        const dfr_options *opt, void *stream, int32_t *tile) {
  dfr_status s = check_single(src, src_h, src_w, src_pitch, src_wcs, tgt_wcs, out_h, out_w,
                              (int)interp);
  if (s != DFR_OK) return s;
  dfr_options o;
  if ((s = resolve_options(opt, o)) != DFR_OK) return s;
  if (!is_f32(o)) return DFR_E_UNSUPPORTED;
  if (out_h == 0 || out_w == 0 || src_h == 0 || src_w == 0) {
    if (tile) *tile = kDefaultTile;
    return DFR_OK;
  }
  if (!out) return DFR_E_NULL;
  o.debug_positions = nullptr;
  FramePlan P;
  build_plan(src, src_h, src_w, src_pitch, *src_wcs, *tgt_wcs, out_h, out_w, out, footprint, P);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // the models do not depend on the tile: computed once, the tile kernels timed
  std::lock_guard<std::mutex> lk(workspace_mutex());
  if ((s = models_for(P, out_h, out_w, o, st)) != DFR_OK) return s;
  auto run = [&](int t) -> bool {
    TileGeom G;
    TileShape ts;
    make_geom(P, out_h, out_w, (int)interp, t, o, G, ts);
    return launch_forward_f32(P, G, (int)interp, ts.np, st) == hipSuccess;
  };
  int best = 0;
  s = time_candidates(run, st, best);
  if (s != DFR_OK) return s;
  tune_store(tune_key(P, out_h, out_w, (int)interp, false), best);
  if (tile) *tile = best;
  return DFR_OK;
}

dfr_status dfr_autotune_batch(int32_t n, const dfr_frame *frames, const dfr_wcs *tgt_wcs,
                              int32_t out_h, int32_t out_w, dfr_interp interp,
                              float *const *outs, float *const *footprints,
                              const dfr_options *opt, void *stream, int32_t *tile) {
  std::vector<FramePlan> plans;
  int t0 = 0, np = 0, max_sord = 0;
  TileGeom G;
  dfr_status s = prepare_batch(n, frames, tgt_wcs, out_h, out_w, (int)interp, outs, footprints,
                               opt, plans, G, t0, np, max_sord);
  if (s != DFR_OK) return s;
  if (plans.empty() || G.n_tiles == 0) {
    if (tile) *tile = kDefaultTile;
    return DFR_OK;
  }
  dfr_options o;
  resolve_options(opt, o);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  auto run = [&](int t) -> bool {
    TileGeom Gt;
    int npt = 0;
    batch_geom(plans, out_h, out_w, (int)interp, t, o, Gt, npt);
    return run_batch(plans, Gt, (int)interp, npt, max_sord, o.precision == DFR_PREC_F32, st,
                     false) == DFR_OK;
  };
  int best = 0;
  s = time_candidates(run, st, best);
  if (s != DFR_OK) return s;
  tune_store(batch_key(plans, out_h, out_w, (int)interp, max_sord), best);
  if (tile) *tile = best;
  return DFR_OK;
}

dfr_status dfr_release(void) {
  release_workspaces();
  return DFR_OK;
}

int64_t dfr_wcs_grad_size(const dfr_wcs *w) {
  if (!w) return 0;
  int64_t na = w->ap_order > 0 ? (int64_t)(w->ap_order + 1) * (w->ap_order + 1) : 0;
  int64_t nb = w->bp_order > 0 ? (int64_t)(w->bp_order + 1) * (w->bp_order + 1) : 0;
  return 8 + na + nb;
}

int32_t dfr_tile_count(void) { return kTileCount; }

dfr_status dfr_tile_shape(int32_t tile, int32_t *width, int32_t *height) {
  TileShape s;
  if (!tile_shape(tile, s)) return DFR_E_ARG;
  if (width) *width = s.width;
  if (height) *height = s.height;
  return DFR_OK;
}

void dfr_cd_from_pc_cdelt(const double pc[4], const double cdelt[2], double cd[4]) {
  if (!pc || !cdelt || !cd) return;
  cd[0] = cdelt[0] * pc[0];
  cd[1] = cdelt[0] * pc[1];
  cd[2] = cdelt[1] * pc[2];
  cd[3] = cdelt[1] * pc[3];
}

dfr_status dfr_cell_model(const dfr_wcs *src_wcs, const dfr_wcs *tgt_wcs, int32_t cx, int32_t cy,
                          double coef_x[10], double coef_y[10], int32_t base[2], double *bound,
                          int32_t *certified, double *tie) {
  if (!src_wcs || !tgt_wcs) return DFR_E_NULL;
  if (cx < 0 || cy < 0 || cx >= (1 << 25) || cy >= (1 << 25)) return DFR_E_ARG;
  dfr_status s;
  if ((s = check_wcs(src_wcs, true)) != DFR_OK) return s;
  if ((s = check_wcs(tgt_wcs, false)) != DFR_OK) return s;
  FramePlan P;
  build_plan(nullptr, 0, 0, 0, *src_wcs, *tgt_wcs, (cy + 1) * kCell, (cx + 1) * kCell, nullptr,
             nullptr, P);
  CellModel M;
  cell_model<-1>(P, cx, cy, M);
  for (int k = 0; k < 10; ++k) {
    if (coef_x) coef_x[k] = M.mx[k];
    if (coef_y) coef_y[k] = M.my[k];
  }
  if (base) {
    base[0] = M.bx;
    base[1] = M.by;
  }
  if (bound) *bound = M.err;
  if (certified) *certified = M.certified;
  if (tie) *tie = M.tie;
  return DFR_OK;
}

dfr_status dfr_check_wcs(const dfr_wcs *wcs, int32_t as_source) {
  return check_wcs(wcs, as_source != 0);
}

const char *dfr_strerror(dfr_status s) {
  switch (s) {
    case DFR_OK: return "success";
    case DFR_E_NULL: return "a required pointer is NULL";
    case DFR_E_SHAPE: return "invalid image shape or pitch";
    case DFR_E_WCS: return "invalid WCS (non-finite value, singular CD, |Dec| > 90, or bad SIP)";
    case DFR_E_UNSUPPORTED: return "unsupported interpolation, precision or WCS form";
    case DFR_E_DEVICE: return "HIP runtime or kernel launch failure";
    case DFR_E_NOMEM: return "out of memory";
    case DFR_E_ARG: return "invalid argument";
    case DFR_E_LIMIT: return "size beyond the fixed limit of the call (static scratch)";
  }
  return "unknown status";
}

int32_t dfr_abi_version(void) { return DFR_ABI_VERSION; }

}  // extern "C"
