// Batched rounds over many views: one update per view per round, every
// level step of all views issued as one multi-view launch per level rank
// (lv_round.h), and the whole round captured once into a HIP graph that each
// round replays.  Workspace: per-view input staging (n_pad x r_max for U and
// for V), then the round's descriptor tables.
#include "lv_round.h"

#include <new>

using namespace lv;

namespace {

lv_status check_views(lv_view* const* views, int count, lv_mode* mode) {
  if (!views || count < 1) return fail(LV_EINVAL, "need at least one view");
  for (int i = 0; i < count; ++i)
    if (!views[i]) return fail(LV_EINVAL, "view %d is NULL", i);
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
  std::vector<lv_view*> views;
  lv_mode mode;
  char* base;
  BatchLayout bl;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

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
  // zero the staging buffers, upload the descriptors
  st = hip_check(hipMemsetAsync(b->base, 0, b->bl.stage_bytes, s), "clear staging");
  if (st == LV_OK)
    st = hip_check(hipMemcpyAsync(b->base + b->bl.stage_bytes, b->bl.plan.bytes.data(), b->bl.plan.bytes.size(),
                                  hipMemcpyHostToDevice, s), "upload descriptors");
  if (st == LV_OK) st = hip_check(hipStreamSynchronize(s), "sync");
  // capture one round on a private stream
  if (st == LV_OK) st = hip_check(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "create capture stream");
  if (st == LV_OK) st = hip_check(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed), "begin capture");
  if (st == LV_OK) {
    const char* dbase = b->base + b->bl.stage_bytes;
    lv_status est = mode == LV_FP64 ? enqueue_round<double>(b->bl.plan, dbase, b->cap)
                                    : enqueue_round<float>(b->bl.plan, dbase, b->cap);
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

lv_status lv_batch_update(lv_batch* b, void* stream) {
  g_err[0] = 0;
  if (!b) return fail(LV_EINVAL, "batch is NULL");
  lv_status st = hip_check(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)), "graph launch");
  if (st == LV_OK)
    for (lv_view* v : b->views) v->updates += 1;
  return st;
}

}  // extern "C"
