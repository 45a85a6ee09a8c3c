// Batched rounds over many views: one update per view per round, every
// level step of all views issued as one multi-view launch per level rank,
// and the whole round captured once into a HIP graph that each round
// replays.
//
// Round order (per level step j, views whose top level is j take the
// update-only pass in the same step):
//   prep (stage -> factor slab 0, all views)
//   for j = 0..max_m:
//     fused passes (R <= 16), one launch per R
//     read-only skinny chunks (R > 16), one launch for all views
//     Gram (R > 16), one launch per R
//     rank-R update of level j (R > 16) and top-level updates, one per R
//     tails (reductions + next factors), one launch per R
// Every view therefore runs exactly the kernels of lv_view_update, so its
// result is identical bit for bit.
#include "lv_view_impl.h"

#include <cstring>
#include <map>
#include <new>
#include <vector>

using namespace lv;

namespace {

enum Kind { kPrep, kFused, kChunk, kGram, kUpdate, kTail };

struct LaunchRec {
  Kind kind;
  int R;
  size_t off;   // byte offset of the descriptor array in the descriptor area
  int nd;
  int blocks;
};

// Host-side plan: descriptor bytes and the launch list.
struct Plan {
  std::vector<char> bytes;
  std::vector<LaunchRec> launches;
  std::vector<size_t> stage_off;   // per view: U staging offset (V follows)
  size_t stage_bytes = 0;
  size_t desc_off = 0;             // start of the descriptor area in the workspace
  size_t total = 0;

  template <typename D, typename F>
  void add(Kind kind, int R, std::vector<D>& ds, F blocks_of) {
    if (ds.empty()) return;
    int b = 0;
    for (auto& d : ds) { d.block_begin = b; b += blocks_of(d); }
    const size_t off = align_up(bytes.size());
    bytes.resize(off + ds.size() * sizeof(D));
    std::memcpy(bytes.data() + off, ds.data(), ds.size() * sizeof(D));
    launches.push_back({kind, R, off, (int)ds.size(), b});
  }
};

template <typename T> int fused_blocks(const FusedDesc<T>& d) {
  return d.nct * ((d.n_pad + d.tile_rows - 1) / d.tile_rows);
}
template <typename T> int update_blocks(const UpdateDesc<T>& d) {
  return d.nct * ((d.n_pad + d.tile_rows - 1) / d.tile_rows);
}
template <typename T> int prep_blocks(const PrepDesc<T>& d) {
  return (int)((d.n_pad * d.r_pad + 255) / 256);
}

template <typename T>
Plan make_plan(const std::vector<lv_view*>& views, char* base) {
  Plan pl;
  size_t off = 0;
  for (lv_view* v : views) {
    pl.stage_off.push_back(off);
    const size_t one = (size_t)v->L.n_pad * v->r_max * sizeof(T);
    off = align_up(off + one);
    off = align_up(off + one);
  }
  pl.stage_bytes = off;
  pl.desc_off = off;
  auto stageU = [&](size_t i) { return reinterpret_cast<const T*>(base + pl.stage_off[i]); };
  auto stageV = [&](size_t i) {
    const size_t one = (size_t)views[i]->L.n_pad * views[i]->r_max * sizeof(T);
    return reinterpret_cast<const T*>(base + pl.stage_off[i] + align_up(one));
  };

  std::vector<PrepDesc<T>> prep;
  int max_m = 0;
  for (size_t i = 0; i < views.size(); ++i) {
    lv_view* v = views[i];
    const Layout& L = v->L;
    prep.push_back({stageU(i), v->r_max, stageV(i), v->r_max, v->n, v->r_max, L.r_pad, v->slabU<T>(0),
                    v->slabV<T>(0), L.W, L.n_pad, 0});
    max_m = L.m > max_m ? L.m : max_m;
  }
  pl.add(kPrep, 0, prep, &prep_blocks<T>);

  for (int j = 0; j <= max_m; ++j) {
    std::map<int, std::vector<FusedDesc<T>>> fused;
    std::vector<FusedDesc<T>> chunks;
    std::map<int, std::vector<GramDesc<T>>> gram;
    std::map<int, std::vector<UpdateDesc<T>>> upd;
    std::map<int, std::vector<TailDesc<T>>> tail;
    for (lv_view* v : views) {
      const Layout& L = v->L;
      if (j > L.m) continue;
      const int R = L.r_pad << j;
      T* sU = v->slabU<T>(0);
      T* sV = v->slabV<T>(0);
      const T* Vj = sV + (L.W - R);
      if (j == L.m) {
        upd[R].push_back({v->P<T>(j), L.ldp, (int)L.n_pad, kUpdateTileRows, sU, Vj, L.W,
                          (int)(L.n_pad / tile_cols_bytes(L.elem)), 0});
        continue;
      }
      if (R <= kMaxFusedRank) {
        fused[R].push_back({v->P<T>(j), L.ldp, (int)L.n_pad, L.tile_rows, sU, Vj, L.W, v->partX<T>(j),
                            v->partY<T>(j), v->partG(j), R, L.nct, 0});
      } else {
        for (int c0 = 0; c0 < R; c0 += kMaxFusedRank)
          chunks.push_back({v->P<T>(j), L.ldp, (int)L.n_pad, L.tile_rows, sU + c0, Vj + c0, L.W,
                            v->partX<T>(j) + c0, v->partY<T>(j) + c0, nullptr, R, L.nct, 0});
        gram[R].push_back({sU, Vj, L.W, (int)L.n_pad, L.tile_rows, v->partG(j), L.nrt, 0});
        upd[R].push_back({v->P<T>(j), L.ldp, (int)L.n_pad, kUpdateTileRows, sU, Vj, L.W,
                          (int)(L.n_pad / tile_cols_bytes(L.elem)), 0});
      }
      tail[R].push_back({v->partX<T>(j), v->partY<T>(j), v->partG(j), L.nct, L.nrt, (int)L.n_pad, sU, sV, L.W, 0});
    }
    for (auto& kv : fused) pl.add(kFused, kv.first, kv.second, &fused_blocks<T>);
    pl.add(kChunk, kMaxFusedRank, chunks, &fused_blocks<T>);
    for (auto& kv : gram) {
      const int R = kv.first;
      const int chunks_per_tile = (R * R + gram_pairs_per_block(R) - 1) / gram_pairs_per_block(R);
      pl.add(kGram, R, kv.second, [chunks_per_tile](const GramDesc<T>& d) { return d.nrt * chunks_per_tile; });
    }
    for (auto& kv : upd) pl.add(kUpdate, kv.first, kv.second, &update_blocks<T>);
    for (auto& kv : tail) {
      const int R = kv.first;
      pl.add(kTail, R, kv.second, [R](const TailDesc<T>& d) { return tail_blocks(d.n_pad, R); });
    }
  }
  pl.total = align_up(pl.desc_off + pl.bytes.size());
  return pl;
}

template <typename T>
lv_status enqueue_round(const Plan& pl, char* base, hipStream_t s) {
  const char* dbase = base + pl.desc_off;
  for (const LaunchRec& l : pl.launches) {
    const void* d = dbase + l.off;
    hipError_t e = hipSuccess;
    switch (l.kind) {
      case kPrep: e = launch_prep_multi<T>(static_cast<const PrepDesc<T>*>(d), l.nd, l.blocks, s); break;
      case kFused: e = launch_fused_multi<T>(l.R, false, static_cast<const FusedDesc<T>*>(d), l.nd, l.blocks, s); break;
      case kChunk: e = launch_fused_multi<T>(l.R, true, static_cast<const FusedDesc<T>*>(d), l.nd, l.blocks, s); break;
      case kGram: e = launch_gram_multi<T>(l.R, static_cast<const GramDesc<T>*>(d), l.nd, l.blocks, s); break;
      case kUpdate: e = launch_update_multi<T>(l.R, static_cast<const UpdateDesc<T>*>(d), l.nd, l.blocks, s); break;
      case kTail: e = launch_tail_multi<T>(l.R, static_cast<const TailDesc<T>*>(d), l.nd, l.blocks, s); break;
    }
    lv_status st = hip_check(e, "batch launch");
    if (st != LV_OK) return st;
  }
  return LV_OK;
}

lv_status check_views(lv_view* const* views, int count, lv_mode* mode) {
  if (!views || count < 1) return fail(LV_EINVAL, "need at least one view");
  for (int i = 0; i < count; ++i)
    if (!views[i]) return fail(LV_EINVAL, "view %d is NULL", i);
  *mode = views[0]->mode;
  for (int i = 1; i < count; ++i)
    if (views[i]->mode != *mode) return fail(LV_EINVAL, "views of different modes in one batch");
  return LV_OK;
}

Plan plan_for(const std::vector<lv_view*>& v, lv_mode mode, char* base) {
  return mode == LV_FP64 ? make_plan<double>(v, base) : make_plan<float>(v, base);
}

}  // namespace

struct lv_batch {
  std::vector<lv_view*> views;
  lv_mode mode;
  char* base;
  Plan plan;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

size_t lv_batch_footprint(lv_view* const* views, int count) {
  lv_mode mode;
  if (check_views(views, count, &mode) != LV_OK) return 0;
  std::vector<lv_view*> v(views, views + count);
  return plan_for(v, mode, nullptr).total;
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
  b->plan = plan_for(b->views, mode, b->base);
  if (ws_bytes < b->plan.total) {
    const size_t need = b->plan.total;
    delete b;
    return fail(LV_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  // zero the staging buffers, upload the descriptors
  st = hip_check(hipMemsetAsync(b->base, 0, b->plan.stage_bytes, s), "clear staging");
  if (st == LV_OK)
    st = hip_check(hipMemcpyAsync(b->base + b->plan.desc_off, b->plan.bytes.data(), b->plan.bytes.size(),
                                  hipMemcpyHostToDevice, s), "upload descriptors");
  if (st == LV_OK) st = hip_check(hipStreamSynchronize(s), "sync");
  // capture one round on a private stream
  if (st == LV_OK) st = hip_check(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "create capture stream");
  if (st == LV_OK) st = hip_check(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed), "begin capture");
  if (st == LV_OK) {
    lv_status est = mode == LV_FP64 ? enqueue_round<double>(b->plan, b->base, b->cap)
                                    : enqueue_round<float>(b->plan, b->base, b->cap);
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
  const size_t es = v->L.elem;
  const size_t one = (size_t)v->L.n_pad * v->r_max * es;
  if (U) *U = b->base + b->plan.stage_off[i];
  if (V) *V = b->base + b->plan.stage_off[i] + align_up(one);
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
