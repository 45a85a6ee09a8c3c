// Serving loop: many views kept on the device inside one caller-provided
// HBM arena, rank-1 update requests from host memory, per-view coalescing of
// queued requests into one rank-r update (the delta of U V^T equals the sum
// of the rank-1 deltas, Sec. 4.1-4.2), and continuous batching: each step
// launches one multi-view round (lv_round.h) over exactly the views that have
// pending requests, without waiting for earlier rounds; requests that arrive
// meanwhile join the next step.  Completion events stamp arrival-to-done
// latency.
//
// Arena layout: kRingSlots descriptor slots at the front, then one block per
// admitted view (its lv_view workspace followed by its device input
// staging, U and V of n_pad x r_coalesce each).  Blocks come from a
// first-fit free list, so admission is exact: a view is admitted only if its
// whole block fits.
#include "lv_round.h"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <new>

using namespace lv;

namespace {

constexpr int kRingSlots = 4;
// Rounds in flight at once: one running, one queued behind it.
constexpr int kMaxInFlight = 2;
constexpr size_t kSlotBytes = 1 << 20;

struct Pending {
  uint64_t ticket;
  double arrival;
  std::vector<char> u, v;
};

struct SView {
  lv_view* view = nullptr;
  size_t off = 0, bytes = 0;
  std::deque<Pending> q;
  char* stage = nullptr;
  bool alive = false;
  // waiting in the admission queue: A (n x n, pinned host memory, read by
  // the creation kernels when the view is admitted), its order and power,
  // and its place in the queue
  bool waiting = false;
  void* hostA = nullptr;
  int64_t n = 0;
  int k = 0;
  uint64_t wait_seq = 0;
};

struct InFlight {
  hipEvent_t ev = nullptr;
  std::vector<std::pair<uint64_t, double>> tickets;
  int slot = 0;
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct lv_server {
  lv_mode mode;
  int elem;
  char* arena;
  size_t arena_bytes;
  int rc;
  int hold_fill = 1;        // hold policy: a view joins a round once it has
  double hold_wait = 0.0;   //   hold_fill requests queued or waited hold_wait s
  hipStream_t stream;
  Lanes lanes;
  std::vector<std::pair<size_t, size_t>> free_blocks;  // (offset, size), sorted by offset
  std::vector<SView> views;
  std::deque<InFlight> inflight;
  char* pinned[kRingSlots] = {};
  size_t pinned_cap[kRingSlots] = {};
  bool slot_busy[kRingSlots] = {};
  uint64_t next_ticket = 1;
  uint64_t submitted = 0, completed = 0, rounds = 0, coalesced_updates = 0;
  bool queue_views = false;      // admission queue on (views wait for arena space)
  uint64_t next_wait_seq = 1, admitted_late = 0;
  std::vector<double> lat;
  std::chrono::steady_clock::time_point t0;
};

namespace {

size_t view_block_bytes(const lv_server* s, int64_t n, int k) {
  const size_t fp = lv_view_footprint(n, k, s->rc, s->mode);
  if (fp == 0) return 0;
  const size_t stage = align_up((size_t)round_up(n, kPadOrder) * s->rc * s->elem);
  return align_up(fp) + 2 * stage;
}

bool arena_alloc(lv_server* s, size_t bytes, size_t* off) {
  for (size_t i = 0; i < s->free_blocks.size(); ++i) {
    auto& b = s->free_blocks[i];
    if (b.second >= bytes) {
      *off = b.first;
      b.first += bytes;
      b.second -= bytes;
      if (b.second == 0) s->free_blocks.erase(s->free_blocks.begin() + (long)i);
      return true;
    }
  }
  return false;
}

void arena_free(lv_server* s, size_t off, size_t bytes) {
  auto& fb = s->free_blocks;
  auto it = std::lower_bound(fb.begin(), fb.end(), std::make_pair(off, (size_t)0));
  it = fb.insert(it, {off, bytes});
  size_t i = (size_t)(it - fb.begin());
  if (i + 1 < fb.size() && fb[i].first + fb[i].second == fb[i + 1].first) {
    fb[i].second += fb[i + 1].second;
    fb.erase(fb.begin() + (long)i + 1);
  }
  if (i > 0 && fb[i - 1].first + fb[i - 1].second == fb[i].first) {
    fb[i - 1].second += fb[i].second;
    fb.erase(fb.begin() + (long)i);
  }
}

size_t largest_free(const lv_server* s) {
  size_t m = 0;
  for (auto& b : s->free_blocks) m = b.second > m ? b.second : m;
  return m;
}

// Create a view in a fresh arena block of `bytes` at `off` from A (device
// or pinned host memory).
lv_status create_in_block(lv_server* s, SView& sv, const void* A, int64_t n, int64_t lda, int k, size_t off,
                          size_t bytes) {
  lv_view* v = nullptr;
  const size_t fp = align_up(lv_view_footprint(n, k, s->rc, s->mode));
  const lv_status st = lv_view_create(A, n, lda, k, s->rc, s->mode, s->arena + off, fp, s->stream, &v);
  if (st != LV_OK) return st;
  sv.view = v;
  sv.off = off;
  sv.bytes = bytes;
  sv.stage = s->arena + off + fp;
  sv.alive = true;
  return LV_OK;
}

// Admit waiting views, in the order they arrived, each one that fits now.
lv_status admit_waiting(lv_server* s) {
  std::vector<int> order;
  for (int i = 0; i < (int)s->views.size(); ++i)
    if (s->views[i].waiting) order.push_back(i);
  std::sort(order.begin(), order.end(),
            [&](int a, int b) { return s->views[a].wait_seq < s->views[b].wait_seq; });
  for (int i : order) {
    SView& sv = s->views[i];
    const size_t bytes = view_block_bytes(s, sv.n, sv.k);
    size_t off = 0;
    if (!arena_alloc(s, bytes, &off)) continue;
    lv_status st = create_in_block(s, sv, sv.hostA, sv.n, sv.n, sv.k, off, bytes);
    if (st == LV_OK) st = hip_check(hipStreamSynchronize(s->stream), "admission");   // host copy of A read
    if (st != LV_OK) {
      arena_free(s, off, bytes);
      return st;
    }
    (void)hipHostFree(sv.hostA);
    sv.hostA = nullptr;
    sv.waiting = false;
    s->admitted_late += 1;
  }
  return LV_OK;
}

// Retire finished rounds (block = wait for the oldest one first).
lv_status retire(lv_server* s, bool block) {
  while (!s->inflight.empty()) {
    InFlight& f = s->inflight.front();
    hipError_t e = block ? hipEventSynchronize(f.ev) : hipEventQuery(f.ev);
    if (e == hipErrorNotReady) return LV_OK;
    if (e != hipSuccess) return fail(LV_EDEVICE, "round completion: %s", hipGetErrorString(e));
    const double t = now_s(s->t0);
    for (auto& tk : f.tickets) s->lat.push_back(t - tk.second);
    s->completed += f.tickets.size();
    s->slot_busy[f.slot] = false;
    (void)hipEventDestroy(f.ev);
    s->inflight.pop_front();
    block = false;
  }
  return LV_OK;
}

int free_slot(lv_server* s) {
  for (int i = 0; i < kRingSlots; ++i)
    if (!s->slot_busy[i]) return i;
  return -1;
}

lv_status wait_all(lv_server* s) {
  while (!s->inflight.empty()) {
    lv_status st = retire(s, true);
    if (st != LV_OK) return st;
  }
  return LV_OK;
}

template <typename T>
lv_status step_impl(lv_server* s, int* launched);

// Apply every queued request: launch rounds (waiting for room as needed)
// until the queues are empty, then wait for every round.
lv_status drain(lv_server* s) {
  for (;;) {
    bool pending = false;
    for (auto& v : s->views) pending = pending || (v.alive && !v.q.empty());
    if (!pending) break;
    int launched = 0;
    lv_status st = s->mode == LV_FP64 ? step_impl<double>(s, &launched) : step_impl<float>(s, &launched);
    if (st != LV_OK) return st;
    if (launched == 0) {
      st = retire(s, true);
      if (st != LV_OK) return st;
    }
  }
  return wait_all(s);
}

template <typename T>
lv_status step_impl(lv_server* s, int* launched) {
  *launched = 0;
  lv_status st = retire(s, false);
  if (st != LV_OK) return st;
  // continuous batching: one round runs while the next waits behind it on
  // the stream; further requests keep coalescing in the queues meanwhile
  if ((int)s->inflight.size() >= kMaxInFlight) return LV_OK;
  std::vector<int> active;
  const double t = now_s(s->t0);
  const int fill = std::min(s->hold_fill, s->rc);
  for (int i = 0; i < (int)s->views.size(); ++i) {
    const SView& sv = s->views[i];
    if (sv.alive && !sv.q.empty() && ((int)sv.q.size() >= fill || t - sv.q.front().arrival >= s->hold_wait))
      active.push_back(i);
  }
  // work-conserving: with no round in flight every pending view goes
  if (active.empty() && s->inflight.empty())
    for (int i = 0; i < (int)s->views.size(); ++i)
      if (s->views[i].alive && !s->views[i].q.empty()) active.push_back(i);
  if (active.empty()) return LV_OK;
  int slot = free_slot(s);
  while (slot < 0) {
    st = retire(s, true);
    if (st != LV_OK) return st;
    slot = free_slot(s);
  }
  // device inputs and the round plan first (the plan needs only device
  // addresses), then one pinned buffer holding the packed factors and the
  // descriptor bytes, alive until the round completes
  std::vector<int> ranks;
  std::vector<lv_view*> views;
  std::vector<RoundInput> in;
  for (int i : active) {
    SView& sv = s->views[i];
    const int r = (int)std::min<size_t>(sv.q.size(), (size_t)s->rc);
    ranks.push_back(r);
    char* dU = sv.stage;
    char* dV = sv.stage + align_up((size_t)sv.view->L.n_pad * s->rc * s->elem);
    views.push_back(sv.view);
    in.push_back({dU, r, dV, r, r});
  }
  Plan pl = make_plan<T>(views, in);
  if (pl.bytes.size() > kSlotBytes) return fail(LV_ENOMEM, "round descriptors exceed %zu bytes", kSlotBytes);
  std::vector<size_t> pin_off;
  size_t need = 0;
  for (size_t a = 0; a < active.size(); ++a) {
    pin_off.push_back(need);
    need += align_up(2 * (size_t)views[a]->n * ranks[a] * sizeof(T));
  }
  const size_t desc_pin = need;
  need += align_up(pl.bytes.size());
  if (need > s->pinned_cap[slot]) {
    if (s->pinned[slot]) (void)hipHostFree(s->pinned[slot]);
    s->pinned[slot] = nullptr;
    s->pinned_cap[slot] = 0;
    if (hipHostMalloc(reinterpret_cast<void**>(&s->pinned[slot]), need, hipHostMallocDefault) != hipSuccess)
      return fail(LV_ENOMEM, "pinned host staging of %zu bytes failed", need);
    s->pinned_cap[slot] = need;
  }
  InFlight f;
  f.slot = slot;
  for (size_t a = 0; a < active.size(); ++a) {
    SView& sv = s->views[active[a]];
    const int64_t n = sv.view->n;
    const int r = ranks[a];
    T* U = reinterpret_cast<T*>(s->pinned[slot] + pin_off[a]);
    T* V = U + (size_t)n * r;
    for (int c = 0; c < r; ++c) {
      const Pending& p = sv.q.front();
      const T* u = reinterpret_cast<const T*>(p.u.data());
      const T* v = reinterpret_cast<const T*>(p.v.data());
      for (int64_t i = 0; i < n; ++i) { U[i * r + c] = u[i]; V[i * r + c] = v[i]; }
      f.tickets.push_back({p.ticket, p.arrival});
      sv.q.pop_front();
    }
    const size_t one = (size_t)n * r * sizeof(T);
    st = hip_check(hipMemcpyAsync(const_cast<void*>(in[a].U), U, one, hipMemcpyHostToDevice, s->stream), "stage U");
    if (st == LV_OK)
      st = hip_check(hipMemcpyAsync(const_cast<void*>(in[a].V), V, one, hipMemcpyHostToDevice, s->stream), "stage V");
    if (st != LV_OK) return st;
  }
  std::memcpy(s->pinned[slot] + desc_pin, pl.bytes.data(), pl.bytes.size());
  char* dslot = s->arena + (size_t)slot * kSlotBytes;
  st = hip_check(hipMemcpyAsync(dslot, s->pinned[slot] + desc_pin, pl.bytes.size(), hipMemcpyHostToDevice, s->stream),
                 "upload descriptors");
  if (st != LV_OK) return st;
  st = enqueue_round<T>(pl, dslot, s->stream, &s->lanes);
  if (st != LV_OK) return st;
  if (hipEventCreateWithFlags(&f.ev, hipEventDisableTiming) != hipSuccess) return fail(LV_EDEVICE, "event create");
  st = hip_check(hipEventRecord(f.ev, s->stream), "event record");
  if (st != LV_OK) return st;
  for (size_t a = 0; a < active.size(); ++a) {
    lv_view* v = s->views[active[a]].view;
    v->updates += 1;
    st = periodic_drift(v, s->stream);   // after the round's completion event
    if (st != LV_OK) return st;
  }
  s->slot_busy[slot] = true;
  *launched = (int)f.tickets.size();
  s->rounds += 1;
  s->coalesced_updates += active.size();
  s->inflight.push_back(std::move(f));
  return LV_OK;
}

}  // namespace

extern "C" {

lv_status lv_server_create(void* arena, size_t arena_bytes, lv_mode mode, int r_coalesce, void* stream,
                           lv_server** out) {
  g_err[0] = 0;
  if (!out) return fail(LV_EINVAL, "out is NULL");
  *out = nullptr;
  if (mode != LV_FP64 && mode != LV_FP32 && mode != LV_FP32_BF16SHADOW) return fail(LV_EINVAL, "unknown mode");
  if (r_coalesce < 1 || r_coalesce > 64) return fail(LV_EINVAL, "r_coalesce outside [1, 64]");
  if (!arena || reinterpret_cast<uintptr_t>(arena) % kAlign) return fail(LV_EINVAL, "arena NULL or misaligned");
  if (arena_bytes < kRingSlots * kSlotBytes) return fail(LV_ENOMEM, "arena smaller than the descriptor ring");
  lv_server* s = new (std::nothrow) lv_server();
  if (!s) return fail(LV_ENOMEM, "host allocation failed");
  s->mode = mode;
  s->elem = mode == LV_FP64 ? 8 : 4;
  s->arena = static_cast<char*>(arena);
  s->arena_bytes = arena_bytes;
  s->rc = r_coalesce;
  s->stream = static_cast<hipStream_t>(stream);
  const lv_status lst = s->lanes.init();
  if (lst != LV_OK) {
    s->lanes.destroy();
    delete s;
    return lst;
  }
  s->free_blocks.push_back({kRingSlots * kSlotBytes, arena_bytes - kRingSlots * kSlotBytes});
  s->t0 = std::chrono::steady_clock::now();
  *out = s;
  return LV_OK;
}

size_t lv_server_view_bytes(const lv_server* s, int64_t n, int k) { return s ? view_block_bytes(s, n, k) : 0; }

lv_status lv_server_set_hold(lv_server* s, int min_fill, double max_wait_s) {
  g_err[0] = 0;
  if (!s) return fail(LV_EINVAL, "server is NULL");
  if (min_fill < 1 || !(max_wait_s >= 0.0)) return fail(LV_EINVAL, "min_fill < 1 or max_wait_s < 0");
  s->hold_fill = min_fill;
  s->hold_wait = max_wait_s;
  return LV_OK;
}

lv_status lv_server_set_admission_queue(lv_server* s, int enable) {
  g_err[0] = 0;
  if (!s) return fail(LV_EINVAL, "server is NULL");
  s->queue_views = enable != 0;
  return LV_OK;
}

lv_status lv_server_add_view(lv_server* s, const void* A, int64_t n, int64_t lda, int k, int* view_id) {
  g_err[0] = 0;
  if (!s || !view_id || !A) return fail(LV_EINVAL, "server, A or view_id is NULL");
  if (lda < n) return fail(LV_EINVAL, "lda < n");
  const size_t bytes = view_block_bytes(s, n, k);
  if (bytes == 0) return fail(LV_EINVAL, "invalid view shape n=%lld k=%d r=%d", (long long)n, k, s->rc);
  SView sv;
  size_t off = 0;
  if (arena_alloc(s, bytes, &off)) {
    const lv_status st = create_in_block(s, sv, A, n, lda, k, off, bytes);
    if (st != LV_OK) { arena_free(s, off, bytes); return st; }
  } else if (!s->queue_views || bytes > s->arena_bytes - kRingSlots * kSlotBytes) {
    return fail(LV_ENOMEM, "admission: view needs %zu bytes, largest free block is %zu", bytes, largest_free(s));
  } else {
    // wait for arena space: keep A in pinned host memory until admission
    const size_t abytes = (size_t)n * n * s->elem;
    void* h = nullptr;
    if (hipHostMalloc(&h, abytes, hipHostMallocDefault) != hipSuccess)
      return fail(LV_ENOMEM, "pinned host copy of A (%zu bytes) for the admission queue failed", abytes);
    lv_status st = hip_check(hipMemcpy2DAsync(h, (size_t)n * s->elem, A, (size_t)lda * s->elem, (size_t)n * s->elem,
                                              (size_t)n, hipMemcpyDeviceToHost, s->stream), "copy A to the host");
    if (st == LV_OK) st = hip_check(hipStreamSynchronize(s->stream), "copy A to the host");
    if (st != LV_OK) { (void)hipHostFree(h); return st; }
    sv.waiting = true;
    sv.hostA = h;
    sv.n = n;
    sv.k = k;
    sv.wait_seq = s->next_wait_seq++;
  }
  int id = -1;
  for (int i = 0; i < (int)s->views.size(); ++i)
    if (!s->views[i].alive && !s->views[i].waiting && s->views[i].view == nullptr) { id = i; break; }
  if (id < 0) { id = (int)s->views.size(); s->views.push_back(std::move(sv)); }
  else s->views[id] = std::move(sv);
  *view_id = id;
  return LV_OK;
}

lv_status lv_server_remove_view(lv_server* s, int id) {
  g_err[0] = 0;
  if (!s || id < 0 || id >= (int)s->views.size() || !(s->views[id].alive || s->views[id].waiting))
    return fail(LV_EINVAL, "no such view");
  if (s->views[id].waiting) {   // never admitted: drop it and its queued requests
    SView& sv = s->views[id];
    s->submitted -= sv.q.size();
    (void)hipHostFree(sv.hostA);
    sv = SView();
    return LV_OK;
  }
  lv_status st = drain(s);
  if (st != LV_OK) return st;
  SView& sv = s->views[id];
  lv_view_destroy(sv.view);
  arena_free(s, sv.off, sv.bytes);
  sv = SView();
  return admit_waiting(s);
}

lv_view* lv_server_view(lv_server* s, int id) {
  if (!s || id < 0 || id >= (int)s->views.size() || !s->views[id].alive) return nullptr;
  return s->views[id].view;
}

double lv_server_now(const lv_server* s) { return s ? now_s(s->t0) : 0.0; }

lv_status lv_server_submit(lv_server* s, int id, const void* u, const void* v, double arrival, uint64_t* ticket) {
  if (!s || id < 0 || id >= (int)s->views.size() || !(s->views[id].alive || s->views[id].waiting))
    return fail(LV_EINVAL, "no such view");
  if (!u || !v) return fail(LV_EINVAL, "u or v is NULL");
  SView& sv = s->views[id];
  const size_t bytes = (size_t)(sv.alive ? sv.view->n : sv.n) * s->elem;
  Pending p;
  p.ticket = s->next_ticket++;
  p.arrival = arrival >= 0.0 ? arrival : now_s(s->t0);
  p.u.assign(static_cast<const char*>(u), static_cast<const char*>(u) + bytes);
  p.v.assign(static_cast<const char*>(v), static_cast<const char*>(v) + bytes);
  if (ticket) *ticket = p.ticket;
  sv.q.push_back(std::move(p));
  s->submitted += 1;
  return LV_OK;
}

lv_status lv_server_step(lv_server* s, int* launched) {
  g_err[0] = 0;
  if (!s) return fail(LV_EINVAL, "server is NULL");
  int dummy = 0;
  return s->mode == LV_FP64 ? step_impl<double>(s, launched ? launched : &dummy)
                            : step_impl<float>(s, launched ? launched : &dummy);
}

lv_status lv_server_drain(lv_server* s) {
  if (!s) return fail(LV_EINVAL, "server is NULL");
  return drain(s);
}

lv_status lv_server_poll(lv_server* s, uint64_t* completed) {
  if (!s) return fail(LV_EINVAL, "server is NULL");
  lv_status st = retire(s, false);
  if (completed) *completed = s->completed;
  return st;
}

lv_status lv_server_stats(const lv_server* s, lv_server_counters* out) {
  if (!s || !out) return fail(LV_EINVAL, "server or out is NULL");
  std::memset(out, 0, sizeof(*out));
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->rounds = s->rounds;
  out->coalesced_updates = s->coalesced_updates;
  int nv = 0, nw = 0;
  for (auto& v : s->views) {
    nv += v.alive ? 1 : 0;
    nw += v.waiting ? 1 : 0;
  }
  out->views = nv;
  out->views_waiting = nw;
  out->admitted_late = s->admitted_late;
  out->arena_free = 0;
  for (auto& b : s->free_blocks) out->arena_free += b.second;
  if (!s->lat.empty()) {
    std::vector<double> l = s->lat;
    std::sort(l.begin(), l.end());
    auto pct = [&](double q) { return l[std::min(l.size() - 1, (size_t)(q * (double)(l.size() - 1) + 0.5))]; };
    out->latency_p50_s = pct(0.50);
    out->latency_p99_s = pct(0.99);
    out->latency_max_s = l.back();
  }
  return LV_OK;
}

void lv_server_destroy(lv_server* s) {
  if (!s) return;
  (void)drain(s);
  for (auto& v : s->views) {
    if (v.alive) lv_view_destroy(v.view);
    if (v.hostA) (void)hipHostFree(v.hostA);
  }
  for (int i = 0; i < kRingSlots; ++i)
    if (s->pinned[i]) (void)hipHostFree(s->pinned[i]);
  s->lanes.destroy();
  delete s;
}

}  // extern "C"
