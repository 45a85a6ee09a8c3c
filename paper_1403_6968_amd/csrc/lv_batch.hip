// Batched rounds over many views: one update per view per round, every
// level step of all views issued as one multi-view launch per level rank
// (lv_round.h), the chains of views of different padded rank on parallel
// stream lanes, and the whole round captured once into a HIP graph that each
// round replays.  Workspace: per-view input staging (n_pad x r_max for U and
// for V), then the round's descriptor tables.
//
// Tile autotuner: before capture, the rows per tile of every level pass are
// chosen by timing.  One round with zero inputs runs first; it leaves every
// stored power unchanged (P + 0) and every factor column zero, so that the
// level launches can then be timed in isolation without changing any view.
// For each (level, rank) group of views the candidates 256, 512 and 1024
// rows are timed over the level's launches (pass, Gram, update, tail; the
// partial count follows the tile height); the fastest is stored in the
// views (lv_view_update then uses the same tiles) and in a process-wide
// cache keyed by device architecture, mode, rank and the group's orders.
#include "lv_round.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <new>
#include <string>

using namespace lv;

namespace {

lv_status check_views(lv_view* const* views, int count, lv_mode* mode) {
  if (!views || count < 1) return fail(LV_EINVAL, "need at least one view");
  for (int i = 0; i < count; ++i) {
    if (!views[i]) return fail(LV_EINVAL, "view %d is NULL", i);
    if (views[i]->L.sums) return fail(LV_EINVAL, "view %d maintains sums of powers: not supported in batches", i);
  }
  *mode = views[0]->mode;
  for (int i = 1; i < count; ++i)
    if (views[i]->mode != *mode) return fail(LV_EINVAL, "views of different modes in one batch");
  return LV_OK;
}

struct BatchLayout {
  std::vector<size_t> stage_off;  // per view: U staging (V follows)
  size_t stage_bytes = 0;
  Plan plan;
  size_t total = 0;
};

size_t stage_one(const lv_view* v) { return align_up((size_t)v->L.n_pad * v->r_max * v->L.elem); }

BatchLayout batch_layout(const std::vector<lv_view*>& views, lv_mode mode, char* base) {
  BatchLayout bl;
  size_t off = 0;
  std::vector<RoundInput> in;
  for (lv_view* v : views) {
    bl.stage_off.push_back(off);
    in.push_back({base + off, v->r_max, base + off + stage_one(v), v->r_max, v->r_max});
    off += 2 * stage_one(v);
  }
  bl.stage_bytes = off;
  bl.plan = mode == LV_FP64 ? make_plan<double>(views, in) : make_plan<float>(views, in);
  bl.total = align_up(off + bl.plan.bytes.size());
  return bl;
}

}  // namespace

struct lv_batch {
  int tuned_groups = 0;
  int cache_hits = 0;
  std::vector<lv_view*> views;
  lv_mode mode;
  char* base;
  BatchLayout bl;
  hipStream_t cap = nullptr;
  Lanes lanes;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;

bool is_pass(Kind k) { return k == kFused || k == kChunk || k == kSkinny || k == kSkinnyF32; }

lv_status upload_plan(lv_batch* b, hipStream_t s) {
  lv_status st = hip_check(hipMemcpyAsync(b->base + b->bl.stage_bytes, b->bl.plan.bytes.data(), b->bl.plan.bytes.size(),
                                          hipMemcpyHostToDevice, s), "upload descriptors");
  if (st == LV_OK) st = hip_check(hipStreamSynchronize(s), "sync");
  return st;
}

template <typename T>
lv_status run_launches(const lv_batch* b, int level, hipStream_t s) {
  const char* dbase = b->base + b->bl.stage_bytes;
  Plan one;
  for (const LaunchRec& l : b->bl.plan.launches)
    if (level < 0 || l.level == level) one.launches.push_back(l);
  return enqueue_round<T>(one, dbase, s);
}

template <typename T>
lv_status autotune(lv_batch* b, hipStream_t s) {
  std::vector<RoundInput> in;
  for (size_t i = 0; i < b->views.size(); ++i) {
    lv_view* v = b->views[i];
    char* u = b->base + b->bl.stage_off[i];
    in.push_back({u, v->r_max, u + stage_one(v), v->r_max, v->r_max});
  }
  // a zero round: unchanged powers, all factor columns zero
  lv_status st = run_launches<T>(b, -1, s);
  if (st != LV_OK) return st;
  hipDeviceProp_t prop;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(LV_EDEVICE, "device query failed");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(LV_EDEVICE, "hipEventCreate failed");
  int max_m = 0;
  for (lv_view* v : b->views) max_m = std::max(max_m, v->L.m);
  // tile rows: every multiple of 128 from 256 to 1024 (the allowed range)
  const int cands[] = {256, 384, 512, 640, 768, 896, 1024};
  for (int j = 0; j < max_m && st == LV_OK; ++j) {
    std::map<int, std::vector<lv_view*>> groups;   // level rank -> views with a pass at level j
    for (lv_view* v : b->views)
      if (j < v->L.m) groups[v->L.r_pad << j].push_back(v);
    for (auto& g : groups) {
      // key: architecture, mode, level rank and the group's orders, each
      // rounded up to a power of two (its n bucket)
      std::vector<int64_t> ns;
      for (lv_view* v : g.second) ns.push_back(next_pow2(v->L.n_pad));
      std::sort(ns.begin(), ns.end());
      std::string arch(prop.gcnArchName);
      arch = arch.substr(0, arch.find(':'));
      std::string key = arch + "|m" + std::to_string((int)b->mode) + "|R" + std::to_string(g.first) + "|n";
      for (int64_t n : ns) key += ":" + std::to_string(n);
      int best = -1;
      {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) best = it->second;
      }
      if (best > 0) {
        b->cache_hits += 1;
      } else {
        float best_ms = 0.f;
        std::vector<int> seen_nrt;
        for (int c : cands) {
          // skip a candidate that gives every view the same row-tile count as one already timed
          int sig = 0;
          for (lv_view* v : g.second) sig = sig * 131 + (int)((v->L.n_pad + c - 1) / c);
          if (std::find(seen_nrt.begin(), seen_nrt.end(), sig) != seen_nrt.end()) continue;
          seen_nrt.push_back(sig);
          for (lv_view* v : g.second) v->tile_rows[j] = c;
          b->bl.plan = b->mode == LV_FP64 ? make_plan<double>(b->views, in) : make_plan<float>(b->views, in);
          st = upload_plan(b, s);
          if (st != LV_OK) break;
          float t_min = 0.f;
          for (int rep = 0; rep < 4 && st == LV_OK; ++rep) {
            st = hip_check(hipEventRecord(e0, s), "event");
            if (st == LV_OK) st = run_launches<T>(b, j, s);
            if (st == LV_OK) st = hip_check(hipEventRecord(e1, s), "event");
            if (st == LV_OK) st = hip_check(hipEventSynchronize(e1), "event sync");
            float ms = 0.f;
            if (st == LV_OK) st = hip_check(hipEventElapsedTime(&ms, e0, e1), "event time");
            if (rep > 0 && (t_min == 0.f || ms < t_min)) t_min = ms;   // rep 0 warms up
          }
          if (st != LV_OK) break;
          if (best < 0 || t_min < best_ms) { best = c; best_ms = t_min; }
        }
        if (st != LV_OK) break;
        b->tuned_groups += 1;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = best;
      }
      for (lv_view* v : g.second) v->tile_rows[j] = best;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != LV_OK) return st;
  b->bl.plan = b->mode == LV_FP64 ? make_plan<double>(b->views, in) : make_plan<float>(b->views, in);
  return upload_plan(b, s);
}

}  // namespace

extern "C" {

lv_status lv_tune_cache_save(const char* path) {
  g_err[0] = 0;
  if (!path) return fail(LV_EINVAL, "path is NULL");
  std::map<std::string, int> copy;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    copy = g_tune_cache;
  }
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return fail(LV_EINVAL, "cannot write %s", tmp.c_str());
  std::fprintf(f, "{\n");
  size_t i = 0;
  for (auto& kv : copy)
    std::fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++i < copy.size() ? "," : "");
  std::fprintf(f, "}\n");
  const bool ok = std::fclose(f) == 0;
  if (!ok || std::rename(tmp.c_str(), path) != 0) return fail(LV_EINVAL, "cannot write %s", path);
  return LV_OK;
}

lv_status lv_tune_cache_load(const char* path, int* entries) {
  g_err[0] = 0;
  if (!path) return fail(LV_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(LV_EINVAL, "cannot read %s", path);
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  std::fclose(f);
  // the file is a flat JSON object of "key": tile-rows pairs (as written by
  // lv_tune_cache_save); keys hold no quotes or escapes
  std::map<std::string, int> add;
  size_t pos = text.find('{');
  if (pos == std::string::npos) return fail(LV_EINVAL, "%s: not a JSON object", path);
  for (;;) {
    const size_t q0 = text.find('"', pos + 1);
    if (q0 == std::string::npos) break;
    const size_t q1 = text.find('"', q0 + 1);
    const size_t colon = q1 == std::string::npos ? q1 : text.find(':', q1 + 1);
    if (colon == std::string::npos) return fail(LV_EINVAL, "%s: malformed entry", path);
    char* end = nullptr;
    const long rows = std::strtol(text.c_str() + colon + 1, &end, 10);
    if (end == text.c_str() + colon + 1 || rows < kMinTileRows || rows > kMaxTileRows || rows % 64 != 0)
      return fail(LV_EINVAL, "%s: bad tile rows for %s", path, text.substr(q0 + 1, q1 - q0 - 1).c_str());
    add[text.substr(q0 + 1, q1 - q0 - 1)] = (int)rows;
    pos = (size_t)(end - text.c_str());
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto& kv : add) g_tune_cache[kv.first] = kv.second;
  }
  if (entries) *entries = (int)add.size();
  return LV_OK;
}

void lv_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache.clear();
}

size_t lv_batch_footprint(lv_view* const* views, int count) {
  lv_mode mode;
  if (check_views(views, count, &mode) != LV_OK) return 0;
  std::vector<lv_view*> v(views, views + count);
  return batch_layout(v, mode, nullptr).total;
}

void lv_batch_destroy(lv_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  b->lanes.destroy();
  delete b;
}

lv_status lv_batch_create(lv_view* const* views, int count, void* workspace, size_t ws_bytes, void* stream,
                          lv_batch** out) {
  g_err[0] = 0;
  if (!out) return fail(LV_EINVAL, "out is NULL");
  *out = nullptr;
  lv_mode mode;
  lv_status st = check_views(views, count, &mode);
  if (st != LV_OK) return st;
  if (!workspace) return fail(LV_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(LV_ENOMEM, "workspace is not %zu-byte aligned", kAlign);
  lv_batch* b = new (std::nothrow) lv_batch();
  if (!b) return fail(LV_ENOMEM, "host allocation failed");
  b->views.assign(views, views + count);
  b->mode = mode;
  b->base = static_cast<char*>(workspace);
  b->bl = batch_layout(b->views, mode, b->base);
  if (ws_bytes < b->bl.total) {
    const size_t need = b->bl.total;
    delete b;
    return fail(LV_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  // zero the staging buffers, upload the descriptors, tune the tiles
  st = hip_check(hipMemsetAsync(b->base, 0, b->bl.stage_bytes, s), "clear staging");
  if (st == LV_OK) st = upload_plan(b, s);
  if (st == LV_OK) st = mode == LV_FP64 ? autotune<double>(b, s) : autotune<float>(b, s);
  // capture one round on a private stream
  if (st == LV_OK) st = hip_check(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "create capture stream");
  if (st == LV_OK) st = b->lanes.init();
  if (st == LV_OK) st = hip_check(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed), "begin capture");
  if (st == LV_OK) {
    const char* dbase = b->base + b->bl.stage_bytes;
    lv_status est = mode == LV_FP64 ? enqueue_round<double>(b->bl.plan, dbase, b->cap, &b->lanes)
                                    : enqueue_round<float>(b->bl.plan, dbase, b->cap, &b->lanes);
    lv_status cst = hip_check(hipStreamEndCapture(b->cap, &b->graph), "end capture");
    st = est != LV_OK ? est : cst;
  }
  if (st == LV_OK) st = hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "instantiate");
  if (st != LV_OK) { lv_batch_destroy(b); return st; }
  *out = b;
  return LV_OK;
}

lv_status lv_batch_inputs(const lv_batch* b, int i, void** U, void** V, int64_t* ld) {
  if (!b || i < 0 || i >= (int)b->views.size()) return fail(LV_EINVAL, "bad batch or view index");
  const lv_view* v = b->views[i];
  if (U) *U = b->base + b->bl.stage_off[i];
  if (V) *V = b->base + b->bl.stage_off[i] + stage_one(v);
  if (ld) *ld = v->r_max;
  return LV_OK;
}

lv_status lv_batch_stage(lv_batch* b, int i, const void* U, const void* V, int64_t r, int64_t ldu,
                         int64_t ldv, void* stream) {
  g_err[0] = 0;
  if (!b || i < 0 || i >= (int)b->views.size()) return fail(LV_EINVAL, "bad batch or view index");
  const lv_view* v = b->views[i];
  if (r < 0 || r > v->r_max) return fail(LV_EINVAL, "rank r = %lld outside [0, %d]", (long long)r, v->r_max);
  if (r > 0 && (!U || !V || ldu < r || ldv < r)) return fail(LV_EINVAL, "bad U/V for rank %lld", (long long)r);
  void *su = nullptr, *sv = nullptr;
  lv_batch_inputs(b, i, &su, &sv, nullptr);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // copy with zero fill: columns >= r and rows >= n of the staging become 0
  if (b->mode == LV_FP64)
    return hip_check(launch_prep<double>(static_cast<const double*>(U), ldu, static_cast<const double*>(V), ldv,
                                         v->n, (int)r, v->r_max, static_cast<double*>(su),
                                         static_cast<double*>(sv), v->r_max, v->L.n_pad, s), "stage");
  return hip_check(launch_prep<float>(static_cast<const float*>(U), ldu, static_cast<const float*>(V), ldv, v->n,
                                      (int)r, v->r_max, static_cast<float*>(su), static_cast<float*>(sv),
                                      v->r_max, v->L.n_pad, s), "stage");
}

lv_status lv_batch_tuning(const lv_batch* b, int* tuned_groups, int* cache_hits) {
  if (!b) return fail(LV_EINVAL, "batch is NULL");
  if (tuned_groups) *tuned_groups = b->tuned_groups;
  if (cache_hits) *cache_hits = b->cache_hits;
  return LV_OK;
}

lv_status lv_batch_update(lv_batch* b, void* stream) {
  g_err[0] = 0;
  if (!b) return fail(LV_EINVAL, "batch is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  lv_status st = hip_check(hipGraphLaunch(b->exec, s), "graph launch");
  if (st != LV_OK) return st;
  for (lv_view* v : b->views) {
    v->updates += 1;
    st = periodic_drift(v, s);
    if (st != LV_OK) return st;
  }
  return LV_OK;
}

}  // extern "C"
