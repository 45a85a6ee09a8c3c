// Round planner shared by batched rounds and the serving loop: for a set of
// views with one update each, per class of equal padded rank (an independent
// chain, run on its own stream lane), the per-level-step multi-view launches
//   prep (update -> factor slab 0, all views)
//   for j = 0..max_m:
//     fused passes (R <= 16), one launch per R
//     read-only skinny chunks (R > 16), one launch for all views
//     Gram (R > 16), one launch per R
//     rank-R update of level j (R > 16) and top-level updates, one per R
//     tails (reductions + next factors), one launch per R
// Views with bfloat16 shadows run, below their top level, the shadow skinny
// pass (one launch per factor-block count), the Gram and the update that
// rewrites the shadow (one launch per R) in place of the fused pass; float
// views at level ranks from 16 up run the float skinny pass the same way.
// Every view runs exactly the kernels of lv_view_update, so its result is
// identical bit for bit to an update applied alone with the same factors.
#pragma once

#include "lv_view_impl.h"

#include <algorithm>
#include <cstring>
#include <map>
#include <vector>

namespace lv {

enum Kind { kPrep, kFused, kChunk, kSkinny, kSkinnyF32, kGram, kGramSum, kUpdate, kUpdateShadow, kUpdateSplit, kTail };

// Views of equal padded rank form a class whose launches depend only on
// each other; classes run as independent chains on up to kMaxLanes streams.
constexpr int kMaxLanes = 4;

struct LaunchRec {
  Kind kind;
  int lane;     // stream lane (class chain) of the launch; the prep is lane 0
  int level;    // level step of the round (-1: prep)
  int R;
  size_t off;   // byte offset of the descriptor array in the descriptor area
  int nd;
  int blocks;
};

// Host-side plan of a round: descriptor bytes (to be copied to device
// memory) and the launch list referring to offsets in them.
struct Plan {
  std::vector<char> bytes;
  std::vector<LaunchRec> launches;

  int level = -1;   // level step the next add() belongs to
  int lane = 0;     // lane the next add() belongs to
  int lanes = 1;    // lanes used

  template <typename D, typename F>
  void add(Kind kind, int R, std::vector<D>& ds, F blocks_of) {
    if (ds.empty()) return;
    int b = 0;
    for (auto& d : ds) { d.block_begin = b; b += blocks_of(d); }
    const size_t off = align_up(bytes.size());
    bytes.resize(off + ds.size() * sizeof(D));
    std::memcpy(bytes.data() + off, ds.data(), ds.size() * sizeof(D));
    launches.push_back({kind, lane, level, R, off, (int)ds.size(), b});
  }
};

template <typename T> int fused_blocks(const FusedDesc<T>& d) {
  return d.nct * ((d.n_pad + d.tile_rows - 1) / d.tile_rows);
}
template <typename T> int update_blocks(const UpdateDesc<T>& d) {
  return d.nct * ((d.n_pad + d.tile_rows - 1) / d.tile_rows);
}
inline int skinny_blocks(const SkinnyDesc& d) { return d.nct * ((d.n_pad + d.tile_rows - 1) / d.tile_rows); }
template <typename T> int prep_blocks(const PrepDesc<T>& d) {
  return (int)((d.n_pad * d.r_pad + 255) / 256);
}

// The update source of one view in a round: U, V (n x r, leading dims
// ldu, ldv) on the device; r may be below the view's r_max (the factor slab
// is zero-filled up to the view's padded rank).
struct RoundInput {
  const void* U; int64_t ldu; const void* V; int64_t ldv; int r;
};

// Descriptors and launch list of one round over `views`.
template <typename T>
Plan make_plan(const std::vector<lv_view*>& views, const std::vector<RoundInput>& in) {
  Plan pl;
  std::vector<PrepDesc<T>> prep;
  int max_m = 0;
  for (size_t i = 0; i < views.size(); ++i) {
    lv_view* v = views[i];
    const Layout& L = v->L;
    prep.push_back({static_cast<const T*>(in[i].U), in[i].ldu, static_cast<const T*>(in[i].V), in[i].ldv, v->n,
                    in[i].r, L.r_pad, v->slabU<T>(), v->slabV<T>(), L.W, L.n_pad, 0});
    max_m = L.m > max_m ? L.m : max_m;
  }
  pl.add(kPrep, 0, prep, &prep_blocks<T>);
  (void)max_m;

  // one chain of launches per class of equal padded rank, largest first;
  // with fewer classes than lanes, a class is split into parts of about
  // equal work (sum of n_pad^2 (m + 1)) so that every lane has a chain
  std::map<int, std::vector<lv_view*>, std::greater<int>> by_rank;
  for (lv_view* v : views) by_rank[v->L.r_pad].push_back(v);
  const int nparts = by_rank.size() >= (size_t)kMaxLanes ? 1 : kMaxLanes / (int)by_rank.size();
  std::vector<std::vector<lv_view*>> groups;
  for (auto& kv : by_rank) {
    std::vector<lv_view*> vs = kv.second;
    std::stable_sort(vs.begin(), vs.end(), [](const lv_view* a, const lv_view* b) { return a->L.n_pad > b->L.n_pad; });
    const int p = std::min<int>(nparts, (int)vs.size());
    std::vector<std::vector<lv_view*>> parts(p);
    std::vector<double> load(p, 0.0);
    for (lv_view* v : vs) {
      const int t = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      parts[t].push_back(v);
      load[t] += (double)v->L.n_pad * v->L.n_pad * (v->L.m + 1);
    }
    for (auto& g : parts) groups.push_back(std::move(g));
  }
  int ci = 0;
  for (const std::vector<lv_view*>& grp : groups) {
  pl.lane = ci++ % kMaxLanes;
  pl.lanes = pl.lane + 1 > pl.lanes ? pl.lane + 1 : pl.lanes;
  int cmax = 0;
  for (lv_view* v : grp) cmax = v->L.m > cmax ? v->L.m : cmax;
  for (int j = 0; j <= cmax; ++j) {
    pl.level = j;
    std::map<int, std::vector<FusedDesc<T>>> fused;
    std::vector<FusedDesc<T>> chunks;
    std::map<int, std::vector<SkinnyDesc>> skinny, skinny32;
    std::map<int, std::vector<GramDesc<T>>> gram;
    std::vector<GramSumDesc> gsum;
    std::map<int, std::vector<UpdateDesc<T>>> upd, updsh, updsplit;
    std::map<int, std::vector<TailDesc<T>>> tail;
    for (lv_view* v : grp) {
      const Layout& L = v->L;
      if (j > L.m) continue;
      const int R = L.r_pad << j;
      const int trows = j < L.m ? v->tile_rows[j] : 0;
      const int nrt = j < L.m ? v->nrt(j) : 0;
      T* sU = v->slabU<T>();
      T* sV = v->slabV<T>();
      const T* Vj = sV + (L.W - R);
      const int upd_rows = update_tile_rows(R, L.elem);
      const int upd_nct = (int)(L.n_pad / update_tile_cols(R, L.elem));
      if (j == L.m) {
        (v->shadowed() ? updsplit : upd)[R].push_back({v->P<T>(j), L.ldp, (int)L.n_pad, upd_rows, sU, Vj, L.W,
                                                       upd_nct, 0});
        continue;
      }
      if constexpr (sizeof(T) == 4) {
        if (v->shadowed() || skinny_on_mfma(R, 4)) {
          if (v->shadowed()) {
            const int per = R <= 64 ? R : 64;
            for (int c0 = 0; c0 < R; c0 += per)
              skinny[skinny_blocks_for(per)].push_back({v->shadow(j), L.ldp, (int)L.n_pad, trows, sU + c0, Vj + c0,
                                                        L.W, per, v->partX<T>(j) + c0, v->partY<T>(j) + c0, R,
                                                        L.nct, 0});
          } else if (skinny_fuses_update(R)) {
            // the skinny pass applies the update too (class + 2: the fused kernels)
            skinny32[2 + skinny_f32_blocks(R)].push_back({v->P<T>(j), L.ldp, (int)L.n_pad, trows, sU, Vj, L.W, R,
                                                          v->partX<T>(j), v->partY<T>(j), R, L.nct, 0});
          } else {
            const int per = R <= 32 ? R : 32;
            for (int c0 = 0; c0 < R; c0 += per)
              skinny32[skinny_f32_blocks(per)].push_back({v->P<T>(j), L.ldp, (int)L.n_pad, trows, sU + c0,
                                                          Vj + c0, L.W, per, v->partX<T>(j) + c0,
                                                          v->partY<T>(j) + c0, R, L.nct, 0});
          }
          gram[R].push_back({sU, Vj, L.W, (int)L.n_pad, kGramRows, v->partG(j), gram_tiles(L.n_pad), 0});
          gsum.push_back({v->partG(j), gram_tiles(L.n_pad), R * R, 0});
          if (v->shadowed() || !skinny_fuses_update(R))
            (v->shadowed() ? updsh : upd)[R].push_back({v->P<T>(j), L.ldp, (int)L.n_pad, upd_rows, sU, Vj, L.W,
                                                        upd_nct, 0, v->shadowed() ? v->shadow(j) : nullptr});
          tail[R].push_back({v->partX<T>(j), v->partY<T>(j), v->partG(j), L.nct, nrt, (int)L.n_pad, sU, sV, L.W,
                             0, 1});
          continue;
        }
      }
      if (R <= kMaxFusedRank) {
        fused[R].push_back({v->P<T>(j), L.ldp, (int)L.n_pad, trows, sU, Vj, L.W, v->partX<T>(j),
                            v->partY<T>(j), v->partG(j), R, L.nct, 0});
      } else {
        for (int c0 = 0; c0 < R; c0 += kMaxFusedRank)
          chunks.push_back({v->P<T>(j), L.ldp, (int)L.n_pad, trows, sU + c0, Vj + c0, L.W,
                            v->partX<T>(j) + c0, v->partY<T>(j) + c0, nullptr, R, L.nct, 0});
        gram[R].push_back({sU, Vj, L.W, (int)L.n_pad, kGramRows, v->partG(j), gram_tiles(L.n_pad), 0});
        gsum.push_back({v->partG(j), gram_tiles(L.n_pad), R * R, 0});
        upd[R].push_back({v->P<T>(j), L.ldp, (int)L.n_pad, upd_rows, sU, Vj, L.W, upd_nct, 0});
      }
      tail[R].push_back({v->partX<T>(j), v->partY<T>(j), v->partG(j), L.nct, nrt, (int)L.n_pad, sU, sV, L.W, 0,
                         gram_in_pass(R, L.elem) ? nrt : 1});
    }
    for (auto& kv : fused) pl.add(kFused, kv.first, kv.second, &fused_blocks<T>);
    pl.add(kChunk, kMaxFusedRank, chunks, &fused_blocks<T>);
    for (auto& kv : skinny) pl.add(kSkinny, kv.first, kv.second, &skinny_blocks);
    for (auto& kv : skinny32) pl.add(kSkinnyF32, kv.first, kv.second, &skinny_blocks);
    for (auto& kv : gram) {
      const int R = kv.first;
      const int chunks_per_tile = (R * R + gram_pairs_per_block(R) - 1) / gram_pairs_per_block(R);
      pl.add(kGram, R, kv.second, [chunks_per_tile](const GramDesc<T>& d) { return d.nrt * chunks_per_tile; });
    }
    pl.add(kGramSum, 0, gsum, [](const GramSumDesc& d) { return (d.count + 255) / 256; });
    for (auto& kv : upd) pl.add(kUpdate, kv.first, kv.second, &update_blocks<T>);
    for (auto& kv : updsh) pl.add(kUpdateShadow, kv.first, kv.second, &update_blocks<T>);
    for (auto& kv : updsplit) pl.add(kUpdateSplit, kv.first, kv.second, &update_blocks<T>);
    for (auto& kv : tail) {
      const int R = kv.first;
      pl.add(kTail, R, kv.second, [R](const TailDesc<T>& d) { return tail_blocks(d.n_pad, R); });
    }
  }
  }
  return pl;
}

// Streams and events for running the lanes of a round concurrently (fork
// after the prep, join at the end).  Streams at the default priority.
struct Lanes {
  hipStream_t s[kMaxLanes] = {};   // s[0] unused: lane 0 runs on the round's stream
  hipEvent_t fork = nullptr;
  hipEvent_t join[kMaxLanes] = {};

  lv_status init() {
    for (int i = 1; i < kMaxLanes; ++i)
      if (hipStreamCreateWithFlags(&s[i], hipStreamNonBlocking) != hipSuccess)
        return fail(LV_EDEVICE, "lane stream creation failed");
    if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess)
      return fail(LV_EDEVICE, "lane event creation failed");
    for (int i = 0; i < kMaxLanes; ++i)
      if (hipEventCreateWithFlags(&join[i], hipEventDisableTiming) != hipSuccess)
        return fail(LV_EDEVICE, "lane event creation failed");
    return LV_OK;
  }
  void destroy() {
    for (int i = 1; i < kMaxLanes; ++i)
      if (s[i]) (void)hipStreamDestroy(s[i]);
    if (fork) (void)hipEventDestroy(fork);
    for (int i = 0; i < kMaxLanes; ++i)
      if (join[i]) (void)hipEventDestroy(join[i]);
  }
};

// Launch a round whose descriptors are at `dbase` on the device.  With
// `lanes`, lane i > 0 runs on lanes->s[i] after the prep (fork) and the
// round's stream waits for every lane at the end (join); without, every
// launch goes to `s` in plan order.
template <typename T>
lv_status enqueue_round(const Plan& pl, const char* dbase, hipStream_t s0, const Lanes* lanes = nullptr) {
  const bool par = lanes != nullptr && pl.lanes > 1;
  bool forked = false;
  for (const LaunchRec& l : pl.launches) {
    const void* d = dbase + l.off;
    hipStream_t s = s0;
    if (par && l.kind != kPrep) {
      if (!forked) {
        if (hipEventRecord(lanes->fork, s0) != hipSuccess) return fail(LV_EDEVICE, "fork record");
        for (int i = 1; i < pl.lanes; ++i)
          if (hipStreamWaitEvent(lanes->s[i], lanes->fork, 0) != hipSuccess) return fail(LV_EDEVICE, "fork wait");
        forked = true;
      }
      if (l.lane > 0) s = lanes->s[l.lane];
    }
    hipError_t e = hipSuccess;
    switch (l.kind) {
      case kPrep: e = launch_prep_multi<T>(static_cast<const PrepDesc<T>*>(d), l.nd, l.blocks, s); break;
      case kFused: e = launch_fused_multi<T>(l.R, false, static_cast<const FusedDesc<T>*>(d), l.nd, l.blocks, s); break;
      case kChunk: e = launch_fused_multi<T>(l.R, true, static_cast<const FusedDesc<T>*>(d), l.nd, l.blocks, s); break;
      case kGram: e = launch_gram_multi<T>(l.R, static_cast<const GramDesc<T>*>(d), l.nd, l.blocks, s); break;
      case kGramSum: e = launch_gram_sum_multi(static_cast<const GramSumDesc*>(d), l.nd, l.blocks, s); break;
      case kSkinnyF32: e = launch_skinny_f32_multi(l.R, static_cast<const SkinnyDesc*>(d), l.nd, l.blocks, s); break;
      case kSkinny: e = launch_skinny_bf16_multi(l.R, static_cast<const SkinnyDesc*>(d), l.nd, l.blocks, s); break;
      case kUpdate:
        e = launch_update_multi<T>(l.R, false, false, static_cast<const UpdateDesc<T>*>(d), l.nd, l.blocks, s);
        break;
      case kUpdateShadow:
        e = launch_update_multi<T>(l.R, true, true, static_cast<const UpdateDesc<T>*>(d), l.nd, l.blocks, s);
        break;
      case kUpdateSplit:
        e = launch_update_multi<T>(l.R, false, true, static_cast<const UpdateDesc<T>*>(d), l.nd, l.blocks, s);
        break;
      case kTail: e = launch_tail_multi<T>(l.R, static_cast<const TailDesc<T>*>(d), l.nd, l.blocks, s); break;
    }
    lv_status st = hip_check(e, "batch launch");
    if (st != LV_OK) return st;
  }
  if (forked) {
    for (int i = 1; i < pl.lanes; ++i) {
      if (hipEventRecord(lanes->join[i], lanes->s[i]) != hipSuccess) return fail(LV_EDEVICE, "join record");
      if (hipStreamWaitEvent(s0, lanes->join[i], 0) != hipSuccess) return fail(LV_EDEVICE, "join wait");
    }
  }
  return LV_OK;
}


}  // namespace lv
