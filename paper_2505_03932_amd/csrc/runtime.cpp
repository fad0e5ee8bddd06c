// Host runtime: tile choice, the tuned-shape cache (optionally persisted as
// JSON), launch geometry, per-device workspaces.
#include "cell_model.hpp"
#include "runtime.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>

#include "plan.hpp"

namespace dfr {

namespace {

std::mutex g_tune_mutex;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;
uint64_t g_tune_generation = 0;  // bumped whenever g_tune changes

const char *cache_path() {
  const char *p = std::getenv("DFR_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

// The cache file is a flat JSON object {"key": tile, ...}.
void load_cache_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char *path = cache_path();
  if (!path) return;
  FILE *f = std::fopen(path, "rb");
  if (!f) return;
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
  std::fclose(f);
  size_t i = 0;
  while (true) {
    size_t q0 = text.find('"', i);
    if (q0 == std::string::npos) break;
    size_t q1 = text.find('"', q0 + 1);
    if (q1 == std::string::npos) break;
    size_t colon = text.find(':', q1);
    if (colon == std::string::npos) break;
    int v = std::atoi(text.c_str() + colon + 1);
    if (v >= 1 && v <= kTileCount) g_tune[text.substr(q0 + 1, q1 - q0 - 1)] = v;
    i = colon + 1;
  }
}

void save_cache_locked() {
  const char *path = cache_path();
  if (!path) return;
  std::string tmp = std::string(path) + ".tmp";
  FILE *f = std::fopen(tmp.c_str(), "wb");
  if (!f) return;
  std::fprintf(f, "{");
  bool first = true;
  for (auto &kv : g_tune) {
    std::fprintf(f, "%s\n  \"%s\": %d", first ? "" : ",", kv.first.c_str(), kv.second);
    first = false;
  }
  std::fprintf(f, "\n}\n");
  std::fclose(f);
  std::rename(tmp.c_str(), path);
}

int lds_need(const FramePlan &P, int32_t out_h, int32_t out_w, int interp, int tile) {
  TileShape s;
  tile_shape(tile, s);
  return estimate_lds_floats(P, out_h, out_w, s, interp);
}

}  // namespace

std::string tune_key(const FramePlan &P, int32_t out_h, int32_t out_w, int interp, bool batch) {
  double mag = max_magnification(P, out_h, out_w);
  int mb = mag > 0 ? (int)std::lround(std::log2(mag) * 2.0) : -99;
  // rotation class from the map's Jacobian at the frame centre
  double xs0, ys0, xs1, ys1;
  int rb = 0;
  double cx = 0.5 * (out_w - 1), cy = 0.5 * (out_h - 1);
  if (position_f64(P, cx, cy, xs0, ys0) && position_f64(P, cx + 8.0, cy, xs1, ys1)) {
    double ang = std::atan2(std::fabs(ys1 - ys0), std::fabs(xs1 - xs0)) * 180.0 / M_PI;
    rb = (int)(ang / 10.0);
  }
  int sord = std::min(P.s_order, 6);
  char key[128];
  std::snprintf(key, sizeof(key), "%s:i%d:s%d:t%d:m%d:r%d", batch ? "batch" : "single", interp,
                sord, P.t_order > 0 ? 1 : 0, mb, rb);
  return key;
}

std::mutex &tune_mutex_for_batch() { return g_tune_mutex; }

int tuned_tile(const std::string &key) {
  load_cache_locked();
  auto it = g_tune.find(key);
  return it == g_tune.end() ? 0 : it->second;
}

void tune_store(const std::string &key, int tile) {
  std::lock_guard<std::mutex> lk(g_tune_mutex);
  load_cache_locked();
  g_tune[key] = tile;
  ++g_tune_generation;
  save_cache_locked();
}

int choose_tile(const FramePlan &P, int32_t out_h, int32_t out_w, int interp, int requested,
                bool batch, int lds_factor, int pref) {
  if (requested >= 1 && requested <= kTileCount) return requested;
  {
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    load_cache_locked();
    if (!g_tune.empty()) {
      auto it = g_tune.find(tune_key(P, out_h, out_w, interp, batch));
      if (it != g_tune.end()) return it->second;
    }
  }
  // heuristic: the measured default for the kernel and interpolation unless
  // the map turns its source box much larger per output pixel than the
  // 64x32 tile's (a rotated map and a flat tile); then 64x32 when its box
  // fits the LDS budget (or the square 64x64 tile when its box is smaller
  // per output pixel still: 218 against 225 us on the 8192^2 frame rotated
  // by 45 degrees), else the largest tile whose box does
  {
    if (pref < 1 || pref > kTileCount) pref = forward_default_tile(interp);
    TileShape a, b;
    tile_shape(pref, a);
    tile_shape(kDefaultTile, b);
    const double na = lds_need(P, out_h, out_w, interp, pref);
    const double nb = lds_need(P, out_h, out_w, interp, kDefaultTile);
    if (lds_factor * na <= kLdsMaxFloats &&
        na / (a.width * a.height) <= 1.5 * nb / (b.width * b.height))
      return pref;
  }
  const double nb = lds_need(P, out_h, out_w, interp, kDefaultTile);
  if (lds_factor * nb <= kLdsMaxFloats) {
    constexpr int kSquareTile = 6;  // 64 x 64, four rows per thread
    TileShape b, c;
    tile_shape(kDefaultTile, b);
    tile_shape(kSquareTile, c);
    const double nc = lds_need(P, out_h, out_w, interp, kSquareTile);
    if (lds_factor * nc <= kLdsMaxFloats &&
        nc / (c.width * c.height) <= 0.95 * nb / (b.width * b.height))
      return kSquareTile;
    return kDefaultTile;
  }
  const int order[] = {4, 8, 1, 7, 10};
  for (int t : order)
    if (lds_factor * lds_need(P, out_h, out_w, interp, t) <= kLdsMaxFloats) return t;
  return 7;
}

void make_geom(const FramePlan &P, int32_t out_h, int32_t out_w, int interp, int tile,
               const dfr_options &o, TileGeom &G, TileShape &ts, int lds_factor) {
  tile_shape(tile, ts);
  std::memset(&G, 0, sizeof(G));
  G.out_h = out_h;
  G.out_w = out_w;
  G.txt_log2 = ts.txt_log2;
  G.tiles_x = (out_w + ts.width - 1) / ts.width;
  int64_t ty = (out_h + ts.height - 1) / ts.height;
  G.n_tiles = (int32_t)(G.tiles_x * ty);
  int64_t need = (int64_t)lds_factor * estimate_lds_floats(P, out_h, out_w, ts, interp);
  G.lds_cap = need <= kLdsMaxFloats ? (int32_t)need : 0;
  G.cubic_a = (float)o.cubic_a;
  G.nan_outside = o.nan_outside ? 1 : 0;
  G.debug = o.debug_positions;
  G.allow_skip = o.debug_positions ? 0 : 1;
}

// ------------------------------------------------ cached single set-up --

namespace {

struct SetupEntry {
  FramePlan P;
  TileGeom G;
  TileShape ts;
};

std::mutex g_setup_mutex;
std::unordered_map<std::string, SetupEntry> g_setup;
constexpr size_t kSetupCacheMax = 256;

void put_bytes(std::string &k, const void *p, size_t n) {
  k.append(static_cast<const char *>(p), n);
}

void put_wcs(std::string &k, const dfr_wcs &w) {
  put_bytes(k, w.crpix, sizeof(w.crpix));
  put_bytes(k, w.crval, sizeof(w.crval));
  put_bytes(k, w.cd, sizeof(w.cd));
  const int32_t orders[4] = {w.a_order, w.b_order, w.ap_order, w.bp_order};
  put_bytes(k, orders, sizeof(orders));
  const double *coef[4] = {w.a, w.b, w.ap, w.bp};
  for (int i = 0; i < 4; ++i)
    if (orders[i] > 0 && coef[i])
      put_bytes(k, coef[i], sizeof(double) * (orders[i] + 1) * (orders[i] + 1));
}

}  // namespace

void single_setup(const float *src, int32_t src_h, int32_t src_w, int64_t src_pitch,
                  const dfr_wcs &sw, const dfr_wcs &tw, int32_t out_h, int32_t out_w,
                  float *out, float *footprint, int interp, const dfr_options &o, FramePlan &P,
                  TileGeom &G, TileShape &ts, int lds_factor, int pref, bool two_rows) {
  std::string key;
  key.reserve(1024);
  uint64_t gen;
  {
    std::lock_guard<std::mutex> lk(g_tune_mutex);
    load_cache_locked();
    gen = g_tune_generation;
  }
  const int64_t ints[9] = {src_h, src_w, out_h, out_w, interp, o.tile, lds_factor, pref,
                           two_rows ? 1 : 0};
  put_bytes(key, ints, sizeof(ints));
  put_bytes(key, &gen, sizeof(gen));
  put_wcs(key, sw);
  put_wcs(key, tw);
  bool hit = false;
  {
    std::lock_guard<std::mutex> lk(g_setup_mutex);
    auto it = g_setup.find(key);
    if (it != g_setup.end()) {
      P = it->second.P;
      G = it->second.G;
      ts = it->second.ts;
      hit = true;
    }
  }
  if (!hit) {
    build_plan(nullptr, src_h, src_w, src_w, sw, tw, out_h, out_w, nullptr, nullptr, P);
    std::memset(&G, 0, sizeof(G));
    std::memset(&ts, 0, sizeof(ts));
    if (out_h > 0 && out_w > 0) {
      int tile = choose_tile(P, out_h, out_w, interp, o.tile, false, lds_factor, pref);
      TileShape t4;
      if (two_rows && tile_shape(tile, t4) && t4.np == 4) tile -= 1;
      dfr_options base;
      dfr_options_init(&base);
      make_geom(P, out_h, out_w, interp, tile, base, G, ts, lds_factor);
    }
    std::lock_guard<std::mutex> lk(g_setup_mutex);
    if (g_setup.size() >= kSetupCacheMax) g_setup.clear();
    g_setup[key] = SetupEntry{P, G, ts};
  }
  // the per-call parts
  P.src = (src_h > 0 && src_w > 0) ? src : nullptr;
  P.pitch = src_pitch;
  P.out = out;
  P.fp = footprint;
  G.cubic_a = (float)o.cubic_a;
  G.nan_outside = o.nan_outside ? 1 : 0;
  G.debug = o.debug_positions;
  G.allow_skip = o.debug_positions ? 0 : 1;
}

// ------------------------------------------------------------ workspaces --

namespace {
std::mutex g_ws_mutex;
std::map<std::pair<int, void *>, Workspace> g_ws;
}  // namespace

std::mutex &workspace_mutex() { return g_ws_mutex; }

Workspace *workspace(hipStream_t stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  Workspace &w = g_ws[std::make_pair(dev, reinterpret_cast<void *>(stream))];
  w.device = dev;
  w.stream = stream;
  return &w;
}

dfr_status workspace_buffer(Workspace *w, size_t bytes, void **buf) {
  *buf = nullptr;
  if (!w) return DFR_E_DEVICE;
  if (w->cap >= bytes && w->buf) {
    *buf = w->buf;
    return DFR_OK;
  }
  if (w->buf) {
    // work already queued on this stream may still use the old buffer; a
    // failed wait is a device error (the old buffer is kept)
    if (hipStreamSynchronize(w->stream) != hipSuccess) return DFR_E_DEVICE;
    (void)hipFree(w->buf);
    w->buf = nullptr;
    w->cap = 0;
  }
  size_t cap = std::max<size_t>(bytes + bytes / 4, 1 << 20);
  if (hipMalloc(&w->buf, cap) != hipSuccess) {
    w->buf = nullptr;
    return DFR_E_NOMEM;
  }
  w->cap = cap;
  *buf = w->buf;
  return DFR_OK;
}

dfr_status workspace_control(Workspace *w, int **ctl) {
  *ctl = nullptr;
  if (!w) return DFR_E_DEVICE;
  if (!w->ctl) {
    if (hipMalloc(&w->ctl, 256) != hipSuccess) {
      w->ctl = nullptr;
      return DFR_E_NOMEM;
    }
    w->ctl_dirty = true;
  }
  if (w->ctl_dirty) {
    if (launch_zero_i32(w->ctl, 64, w->stream) != hipSuccess) return DFR_E_DEVICE;
    w->ctl_dirty = false;
  }
  *ctl = w->ctl;
  return DFR_OK;
}

namespace {

void destroy_graphs(Workspace &w) {
  for (auto &g : w.graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  w.graphs.clear();
}

}  // namespace

void release_workspaces() {
  std::lock_guard<std::mutex> lk(g_ws_mutex);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  for (auto it = g_ws.begin(); it != g_ws.end();) {
    if (it->first.first != dev) {
      ++it;
      continue;
    }
    Workspace &w = it->second;
    (void)hipStreamSynchronize(w.stream);
    destroy_graphs(w);
    if (w.buf) (void)hipFree(w.buf);
    if (w.ctl) (void)hipFree(w.ctl);
    if (w.host_plans) (void)hipHostFree(w.host_plans);
    if (w.staged) (void)hipEventDestroy(w.staged);
    it = g_ws.erase(it);
  }
}

// ----------------------------------------------------------------- batch --

dfr_status run_batch(const std::vector<FramePlan> &plans, const TileGeom &G, int interp, int np,
                     int max_sord, bool models, hipStream_t stream, bool graph,
                     const BatchRun &run) {
  const CoaddOut *coadd = run.coadd;
  if (coadd || run.crop_items >= 0 || run.reach_host) graph = false;
  std::lock_guard<std::mutex> lk(g_ws_mutex);
  Workspace *w = workspace(stream);
  if (!w) return DFR_E_DEVICE;
  const int n = (int)plans.size();
  const size_t table = (size_t)n * sizeof(FramePlan);
  // counter + reach boxes (4 ints per frame, zeroed together) | frame table |
  // per-frame model tables (when used)
  models = models && plans[0].t_order == 0;
  const int ncx = (G.out_w + kCell - 1) / kCell, ncy = (G.out_h + kCell - 1) / kCell;
  const int64_t ncells = (int64_t)ncx * ncy;
  const int64_t nzero = 4 + 4 * (int64_t)n;  // counter padded to 16 bytes, then the boxes
  const size_t tofs = ((size_t)nzero * 4 + 255) & ~(size_t)255;
  const size_t mofs = (tofs + table + 255) & ~(size_t)255;
  const size_t mbytes = models ? (size_t)n * ncells * sizeof(CellModel) : 0;
  void *wsbuf = nullptr;
  dfr_status ws = workspace_buffer(w, mofs + mbytes, &wsbuf);
  if (ws != DFR_OK) return ws;
  char *dev = static_cast<char *>(wsbuf);
  int *counter = reinterpret_cast<int *>(dev);
  int32_t *reach = reinterpret_cast<int32_t *>(dev) + 4;
  FramePlan *plans_dev = reinterpret_cast<FramePlan *>(dev + tofs);
  CellModel *models_dev = models ? reinterpret_cast<CellModel *>(dev + mofs) : nullptr;
  // the previous batch on this stream must have copied the staged table
  if (w->staged_pending) {
    if (hipEventSynchronize(w->staged) != hipSuccess) return DFR_E_DEVICE;
    w->staged_pending = false;
  }
  if (w->host_cap < (size_t)n) {
    if (w->host_plans) (void)hipHostFree(w->host_plans);
    w->host_plans = nullptr;
    w->host_cap = 0;
    if (hipHostMalloc(reinterpret_cast<void **>(&w->host_plans), table, hipHostMallocDefault) !=
        hipSuccess)
      return DFR_E_NOMEM;
    w->host_cap = n;
  }
  std::memcpy(w->host_plans, plans.data(), table);
  for (int i = 0; i < n; ++i) {
    w->host_plans[i].models = models ? models_dev + i * ncells : nullptr;
    w->host_plans[i].reach = models ? reach + 4 * i : nullptr;
  }
  int dev_id = 0, cus = 0;
  if (hipGetDevice(&dev_id) != hipSuccess) return DFR_E_DEVICE;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id) != hipSuccess ||
      cus < 1)
    cus = 1;
  const int lds_bytes = G.lds_cap * (int)sizeof(float);
  const int grid = batch_blocks_per_cu(interp, np, max_sord, lds_bytes) * cus;
  const int64_t mtotal = (int64_t)n * ncells;
  const dim3 mgrid((unsigned)((mtotal + 63) / 64));
  int ncx_i = ncx, ncells_i = (int)ncells;
  int64_t mtotal_i = mtotal;
  void *margs[] = {&plans_dev, &ncx_i, &ncells_i, &mtotal_i, &models_dev};
  if (!graph) {
    if (hipMemcpyAsync(plans_dev, w->host_plans, table, hipMemcpyHostToDevice, stream) !=
        hipSuccess)
      return DFR_E_DEVICE;
    // counter and reach boxes start at zero; the prepass then records the boxes
    if (launch_zero_i32(counter, nzero, stream) != hipSuccess) return DFR_E_DEVICE;
    if (models && hipLaunchKernel(cell_models_batch_ptr(max_sord), mgrid, dim3(64), margs, 0,
                                  stream) != hipSuccess)
      return DFR_E_DEVICE;
    if (run.reach_host) {
      // the reach boxes the prepass recorded, back to the host (no model
      // table: every frame may reach everywhere, reported as -1); the wait
      // also ends the frame table's copy from the pinned staging buffer,
      // which the next batch on this stream refills
      if (models && hipMemcpyAsync(run.reach_host, reach, (size_t)16 * n, hipMemcpyDeviceToHost,
                                   stream) != hipSuccess)
        return DFR_E_DEVICE;
      if (hipStreamSynchronize(stream) != hipSuccess) return DFR_E_DEVICE;
      if (!models)
        for (int i = 0; i < 4 * n; ++i) run.reach_host[i] = -1;
      return DFR_OK;
    }
    const hipError_t e =
        coadd ? launch_coadd_f32(plans_dev, n, max_sord, G, interp, np, *coadd, stream)
        : run.crop_items >= 0
            ? launch_batch_cropped(plans_dev, n, (int)run.crop_items, max_sord, G, interp, np,
                                   counter, grid, stream)
            : launch_batch_f32(plans_dev, n, max_sord, G, interp, np, counter, grid, stream);
    if (e != hipSuccess) return DFR_E_DEVICE;
  } else {
    BatchGraph *found = nullptr;
    for (auto &g : w->graphs)
      if (g.n == n && g.interp == interp && g.np == np && g.sord == max_sord && g.grid == grid &&
          g.models == (int)models && g.plans_dev == plans_dev && g.plans_host == w->host_plans &&
          std::memcmp(&g.geom, &G, sizeof(G)) == 0)
        found = &g;
    if (!found) {
      BatchGraph bg;
      std::memset(&bg, 0, sizeof(bg));
      bg.geom = G;
      bg.n = n;
      bg.interp = interp;
      bg.np = np;
      bg.sord = max_sord;
      bg.grid = grid;
      bg.models = (int)models;
      bg.plans_dev = plans_dev;
      bg.plans_host = w->host_plans;
      if (hipGraphCreate(&bg.graph, 0) != hipSuccess) return DFR_E_DEVICE;
      hipGraphNode_t copy = nullptr, mod = nullptr, zero = nullptr, kern = nullptr;
      bool ok = hipGraphAddMemcpyNode1D(&copy, bg.graph, nullptr, 0, plans_dev, w->host_plans,
                                        table, hipMemcpyHostToDevice) == hipSuccess;
      if (models) {
        hipKernelNodeParams mp;
        std::memset(&mp, 0, sizeof(mp));
        mp.func = const_cast<void *>(cell_models_batch_ptr(max_sord));
        mp.gridDim = mgrid;
        mp.blockDim = dim3(64);
        mp.sharedMemBytes = 0;
        mp.kernelParams = margs;
        ok = ok && hipGraphAddKernelNode(&mod, bg.graph, &copy, 1, &mp) == hipSuccess;
      }
      int64_t nz = nzero;
      void *zargs[] = {&counter, &nz};
      hipKernelNodeParams zp;
      std::memset(&zp, 0, sizeof(zp));
      zp.func = const_cast<void *>(zero_i32_kernel_ptr());
      zp.gridDim = dim3(1);
      zp.blockDim = dim3(256);
      zp.sharedMemBytes = 0;
      zp.kernelParams = zargs;
      ok = ok && hipGraphAddKernelNode(&zero, bg.graph, nullptr, 0, &zp) == hipSuccess;
      TileGeom geom = G;
      int nf = n;
      void *kargs[] = {&plans_dev, &nf, &geom, &counter};
      hipKernelNodeParams kp;
      std::memset(&kp, 0, sizeof(kp));
      kp.func = const_cast<void *>(batch_kernel_ptr(interp, np, max_sord));
      kp.gridDim = dim3(grid);
      kp.blockDim = dim3(kThreads);
      kp.sharedMemBytes = lds_bytes;
      kp.kernelParams = kargs;
      hipGraphNode_t deps[2] = {models ? mod : copy, zero};
      ok = ok && hipGraphAddKernelNode(&kern, bg.graph, deps, 2, &kp) == hipSuccess;
      // the prepass records the reach boxes: it runs after they are zeroed
      if (models) ok = ok && hipGraphAddDependencies(bg.graph, &zero, &mod, 1) == hipSuccess;
      ok = ok && hipGraphInstantiate(&bg.exec, bg.graph, nullptr, nullptr, 0) == hipSuccess;
      if (!ok) {
        (void)hipGraphDestroy(bg.graph);
        return DFR_E_DEVICE;
      }
      w->graphs.push_back(bg);
      found = &w->graphs.back();
    }
    if (hipGraphLaunch(found->exec, stream) != hipSuccess) return DFR_E_DEVICE;
  }
  if (!w->staged && hipEventCreateWithFlags(&w->staged, hipEventDisableTiming) != hipSuccess)
    return DFR_E_DEVICE;
  if (hipEventRecord(w->staged, stream) != hipSuccess) return DFR_E_DEVICE;
  w->staged_pending = true;
  return DFR_OK;
}

}  // namespace dfr
