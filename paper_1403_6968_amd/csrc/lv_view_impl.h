// Internal view state shared by the C-ABI translation units: workspace
// layout of a view, the view handle, and error helpers.
#pragma once

#include "linview.h"
#include "lv_internal.h"

#include <cstdarg>
#include <cstdio>
#include <vector>

namespace lv {

// Message of the last failure on this host thread (set by fail()).
extern thread_local char g_err[512];
lv_status fail(lv_status st, const char* fmt, ...);

inline bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }
inline int ilog2(int64_t x) { int m = 0; while ((int64_t(1) << m) < x) ++m; return m; }
inline int64_t next_pow2(int64_t x) { int64_t p = 1; while (p < x) p <<= 1; return p; }

constexpr size_t kAlign = 256;
constexpr int64_t kMaxOrder = 65536;
constexpr int kMaxK = 1024;
constexpr int kMaxWidth = 2 * kMaxLevelRank;   // k * r_pad: width of the top-level factors
constexpr int kTileRows = 512;      // default rows per tile of a level pass
constexpr int kMinTileRows = 256;   // tile rows a level pass may be set to:
constexpr int kMaxTileRows = 1024;  //   multiples of 64 in [256, 1024]

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  int64_t n_pad = 0, ldp = 0;
  int m = 0, r_pad = 0, W = 0, elem = 0, nct = 0, nrt_max = 0, tile_rows = 0;
  size_t P[kMaxLevel + 1] = {};
  size_t slabU = 0, slabV = 0;   // the update's factor slabs (every level's U_j, V_j)
  // factor-slab pairs of the pipelined batch (plain views with m >= 2): slot
  // 0 is slabU / slabV, slots 1 .. pipe_slots - 1 follow
  int pipe_slots = 0;
  size_t pslabU[kMaxPipeSlots] = {}, pslabV[kMaxPipeSlots] = {};
  // n_pad x r_pad zeros (set at creation): the factors of the zero updates
  // that lv_view_autotune times (P + 0 0^T = P exactly)
  size_t zfac = 0;
  size_t partX[kMaxLevel] = {};
  size_t partY[kMaxLevel] = {};
  size_t partG[kMaxLevel] = {};
  size_t shadow[kMaxLevel] = {};   // bfloat16 copies of P_0..P_{m-1} (LV_FP32_BF16SHADOW)
  size_t scratch[2] = {};
  // sums of powers (LV_WITH_SUMS): S_1 = I, S_2, ..., S_k, their factor
  // slabs Q (prefix columns) and W (suffix columns), per-level partials of
  // P_j Q_j, S_j^T V_j and the Gram Q_j^T V_j, FP64 squaring scratch
  bool sums = false;
  size_t S[kMaxLevel + 1] = {};
  size_t slabQ = 0, slabW = 0;
  size_t partXs[kMaxLevel] = {};
  size_t partYs[kMaxLevel] = {};
  size_t partGs[kMaxLevel] = {};
  size_t sscratch[2] = {};
  // general form T_{i+1} = A T_i + B with hybrid deltas (implies sums): p
  // columns padded to pp, T_1, T_2, ..., T_k and T_0, B (storage type, n_pad x
  // pp), the deltas D (two, ping-pong), partials of P_j D_j (and of the
  // unused P_j^T D_j), FP64 partials of V_j^T T_j and W_j^T B, FP64 creation
  // scratch (two T, one product, B)
  bool general = false;
  int p = 0, pp = 0;
  // factored deltas Delta T_j = Y_j Z_j^T instead (LV_GENERAL_FACTORED):
  // p padded to a multiple of 128; Y_j slabs (n_pad x WY[j], true width
  // wy[j]; Y_0 is the prefix of the powers' U slab), Z_j kept transposed
  // (WY[j] x pp), FP64 partials of V_j^T Y_j
  bool gfac = false;
  int wy[kMaxLevel + 1] = {};
  int WY[kMaxLevel + 1] = {};
  size_t Y[kMaxLevel + 1] = {};
  size_t Zt[kMaxLevel + 1] = {};
  size_t atbG = 0;
  // skip-s model (factored deltas only): the powers and sums stop at
  // P_s = P_{2^m}; T_{2s}, T_{3s}, ..., T_{kT} follow T_{js} = P_s T_{(j-1)s} + S_s B
  // (nsk of them, uniform strides), with factor slabs of widths wsk(q)
  int kT = 0, nsk = 0;
  size_t Tsk = 0, Ysk = 0, Ztsk = 0, tstride = 0, ystride = 0, zstride = 0;
  int wsk(int q) const { return wy[m] + q * 2 * (r_pad << m); }
  int WYsk(int q) const { return (int)next_pow2(wsk(q)); }
  size_t T[kMaxLevel + 1] = {};
  size_t T0 = 0, B = 0, D[2] = {}, partXT = 0, partYT = 0, atbA = 0, atbB = 0;
  size_t gT[2] = {}, gTmp = 0, gB = 0;
  size_t probe = 0;  // zpad | Pz (m+1 vectors) | PPz (m vectors) | residuals | gate | counter
  size_t drift_z = 0;  // probe vector of the periodic drift check (n_pad doubles)
  size_t total = 0;
};

// wide: a plain float view (FP32 or BF16 shadows, no sums, no general form),
// whose top factors may be kMaxWidth wide; other views stop at
// kMaxLevelRank (their level passes take ranks up to kMaxLevelRank / 2).
inline lv_status check_shape(int64_t n, int k, int r_max, lv_mode mode, bool wide = false) {
  if (mode != LV_FP64 && mode != LV_FP32 && mode != LV_FP32_BF16SHADOW)
    return fail(LV_EINVAL, "unknown mode %d", (int)mode);
  if (n < 1 || n > kMaxOrder) return fail(LV_EINVAL, "n = %lld outside [1, %lld]", (long long)n, (long long)kMaxOrder);
  if (!is_pow2(k) || k > kMaxK) return fail(LV_EINVAL, "k = %d is not a power of two in [1, %d]", k, kMaxK);
  if (r_max < 1) return fail(LV_EINVAL, "r_max = %d < 1", r_max);
  const int64_t width = (int64_t)k * next_pow2(r_max);
  const int cap = wide && mode != LV_FP64 ? kMaxWidth : kMaxLevelRank;
  if (width > cap)
    return fail(LV_EINVAL, "k * r_max (rounded up to a power of two) = %lld exceeds %d", (long long)width, cap);
  return LV_OK;
}

constexpr int kMaxGeneralCols = 64;      // p with hybrid deltas (padded to a power of two)
constexpr int kMaxGeneralColsF = 4096;  // p with factored deltas (padded to a multiple of 128)
constexpr int kMaxGeneralWidthF = 128;  // k * r_pad with factored deltas
constexpr int kAtbRows = 64;          // rows per FP64 partial of V^T T and W^T B

// ext_powers: the stored powers live outside the workspace (the caller's
// buffers); the layout then holds only the factor slabs and the per-level
// partials of an update (the regions a plain update of a FP32 or FP64 view
// touches) and starts with them at offset 0.
inline Layout make_layout(int64_t n, int k, int r_max, lv_mode mode, int flags = 0, int p = 0,
                          bool factored = false, int kT = 0, bool ext_powers = false) {
  lv::Layout L;
  L.general = p > 0;
  L.gfac = L.general && factored;
  L.kT = kT > 0 ? kT : k;
  L.nsk = L.gfac ? L.kT / k - 1 : 0;
  L.sums = (flags & LV_WITH_SUMS) != 0 || L.general;
  L.elem = mode == LV_FP64 ? 8 : 4;
  L.n_pad = round_up(n, kPadOrder);
  L.ldp = L.n_pad;
  L.m = ilog2(k);
  L.r_pad = (int)next_pow2(r_max);
  L.W = k * L.r_pad;
  L.tile_rows = kTileRows;
  L.nct = (int)(L.n_pad / tile_cols_bytes(L.elem));
  L.nrt_max = (int)((L.n_pad + kMinTileRows - 1) / kMinTileRows);   // partials sized for the smallest tiles
  size_t off = 0;
  const size_t mat = (size_t)L.n_pad * L.ldp * L.elem;
  if (!ext_powers)
    for (int j = 0; j <= L.m; ++j) { L.P[j] = off; off = align_up(off + mat); }
  const size_t slab = (size_t)L.n_pad * L.W * L.elem;
  L.slabU = off; off = align_up(off + slab);
  L.slabV = off; off = align_up(off + slab);
  L.pslabU[0] = L.slabU;
  L.pslabV[0] = L.slabV;
  if (!ext_powers && !L.sums && L.m >= 2) {
    L.pipe_slots = L.m + 1 < kMaxPipeSlots ? L.m + 1 : kMaxPipeSlots;
    for (int q = 1; q < L.pipe_slots; ++q) {
      L.pslabU[q] = off; off = align_up(off + slab);
      L.pslabV[q] = off; off = align_up(off + slab);
    }
  }
  if (!ext_powers) {
    L.zfac = off;
    off = align_up(off + (size_t)L.n_pad * L.r_pad * L.elem);
  }
  for (int j = 0; j < L.m; ++j) {
    const size_t R = (size_t)L.r_pad << j;
    L.partX[j] = off; off = align_up(off + (size_t)L.nct * L.n_pad * R * L.elem);
    L.partY[j] = off; off = align_up(off + (size_t)L.nrt_max * L.n_pad * R * L.elem);
    const size_t ng = (size_t)(gram_tiles(L.n_pad) > L.nrt_max ? gram_tiles(L.n_pad) : L.nrt_max);
    L.partG[j] = off; off = align_up(off + ng * R * R * sizeof(double));
  }
  if (ext_powers) {
    L.total = off;
    return L;
  }
  if (mode == LV_FP32_BF16SHADOW)
    for (int j = 0; j < L.m; ++j) { L.shadow[j] = off; off = align_up(off + (size_t)L.n_pad * L.ldp * 2); }
  if (mode != LV_FP64 && (L.m > 0 || L.general)) {
    const size_t dmat = (size_t)L.n_pad * L.n_pad * sizeof(double);
    L.scratch[0] = off; off = align_up(off + dmat);
    L.scratch[1] = off; off = align_up(off + dmat);
  }
  if (L.sums) {
    for (int j = 0; j <= L.m; ++j) { L.S[j] = off; off = align_up(off + mat); }
    L.slabQ = off; off = align_up(off + slab);
    L.slabW = off; off = align_up(off + slab);
    for (int j = 0; j < L.m; ++j) {
      const size_t R = (size_t)L.r_pad << j;
      L.partXs[j] = off; off = align_up(off + (size_t)L.nct * L.n_pad * R * L.elem);
      L.partYs[j] = off; off = align_up(off + (size_t)L.nrt_max * L.n_pad * R * L.elem);
      L.partGs[j] = off; off = align_up(off + (size_t)gram_tiles(L.n_pad) * R * R * sizeof(double));
    }
    if (mode != LV_FP64 && (L.m > 0 || L.general)) {
      const size_t dmat = (size_t)L.n_pad * L.n_pad * sizeof(double);
      L.sscratch[0] = off; off = align_up(off + dmat);
      L.sscratch[1] = off; off = align_up(off + dmat);
    }
  }
  if (L.general) {
    L.p = p;
    L.pp = L.gfac ? (int)round_up(p, 128) : (int)next_pow2(p);
    const size_t gmat = (size_t)L.n_pad * L.pp * L.elem;
    const size_t gdbl = (size_t)L.n_pad * L.pp * sizeof(double);
    for (int j = 0; j <= L.m; ++j) { L.T[j] = off; off = align_up(off + gmat); }
    L.T0 = off; off = align_up(off + gmat);
    L.B = off; off = align_up(off + gmat);
    size_t rmax = (size_t)(L.m > 0 ? L.r_pad << (L.m - 1) : L.r_pad);
    if (L.gfac) {
      L.wy[0] = L.WY[0] = L.r_pad;
      int wmax = L.r_pad;
      for (int j = 1; j <= L.m; ++j) {
        L.wy[j] = 2 * (L.r_pad << (j - 1)) + L.wy[j - 1];
        L.WY[j] = (int)next_pow2(L.wy[j]);
        if (j < L.m && L.WY[j] > wmax) wmax = L.WY[j];
      }
      for (int j = 1; j <= L.m; ++j) { L.Y[j] = off; off = align_up(off + (size_t)L.n_pad * L.WY[j] * L.elem); }
      for (int j = 0; j <= L.m; ++j) { L.Zt[j] = off; off = align_up(off + (size_t)L.WY[j] * L.pp * L.elem); }
      if (L.nsk > 0) {
        rmax = (size_t)(L.r_pad << L.m);
        for (int q = 0; q < L.nsk; ++q) wmax = L.WYsk(q) > wmax ? L.WYsk(q) : wmax;   // widths of the P_s passes
        const int wtop = L.WYsk(L.nsk);
        L.tstride = align_up(gmat);
        L.ystride = align_up((size_t)L.n_pad * wtop * L.elem);
        L.zstride = align_up((size_t)wtop * L.pp * L.elem);
        L.Tsk = off; off += L.nsk * L.tstride;
        L.Ysk = off; off += L.nsk * L.ystride;
        L.Ztsk = off; off += L.nsk * L.zstride;
      }
      const size_t xmat = (size_t)L.n_pad * wmax * L.elem;
      L.partXT = off; off = align_up(off + (size_t)L.nct * xmat);
      L.partYT = off; off = align_up(off + (size_t)L.nrt_max * xmat);
      L.atbG = off; off = align_up(off + (size_t)(L.n_pad / kAtbRows) * rmax * wmax * sizeof(double));
    } else {
      L.D[0] = off; off = align_up(off + gmat);
      L.D[1] = off; off = align_up(off + gmat);
      L.partXT = off; off = align_up(off + (size_t)L.nct * gmat);
      L.partYT = off; off = align_up(off + (size_t)L.nrt_max * gmat);
    }
    const size_t atb = (size_t)(L.n_pad / kAtbRows) * rmax * L.pp * sizeof(double);
    L.atbA = off; off = align_up(off + atb);
    L.atbB = off; off = align_up(off + atb);
    L.gT[0] = off; off = align_up(off + gdbl);
    L.gT[1] = off; off = align_up(off + gdbl);
    L.gTmp = off; off = align_up(off + gdbl);
    L.gB = off; off = align_up(off + gdbl);
  }
  L.probe = off;
  off = align_up(off + (size_t)(2 * L.m + 2) * L.n_pad * sizeof(double) + kMaxLevel * sizeof(double) + 256);
  L.drift_z = off;
  off = align_up(off + (size_t)L.n_pad * sizeof(double));
  L.total = off;
  return L;
}

// The periodic drift check of a view after an update (no-op unless the
// view's update count is a multiple of its interval); stream-ordered on s.
lv_status periodic_drift(::lv_view* v, hipStream_t s);

inline lv_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return LV_OK;
  return fail(LV_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace lv

struct lv_view {
  int64_t n;
  int k;
  int r_max;
  lv_mode mode;
  lv::Layout L;
  char* base;
  size_t ws_bytes;
  int64_t updates;
  int64_t reanchors;
  // periodic drift check: after every drift_every-th update (0: never) with
  // bound drift_tau and the probe vector at L.drift_z; checks enqueued so far
  int64_t drift_every = 0;
  double drift_tau = 0.0;
  int64_t drift_checks = 0;
  // Rows per tile of the level pass of each level below the top (set by the
  // batch autotuner or lv_view_set_tile_rows; every path uses the same value,
  // which fixes the reduction order of the partial sums).
  int tile_rows[lv::kMaxLevel];
  int nrt(int j) const { return (int)((L.n_pad + tile_rows[j] - 1) / tile_rows[j]); }

  // Kernel timing (diagnostics): event pairs per launch kind, resolved by
  // lv_view_timing.
  bool timing = false;
  struct Pair { hipEvent_t a, b; int kind; };
  std::vector<Pair> pending;
  std::vector<hipEvent_t> pool;

  // Pipelined update_batch (plain views, L.pipe_slots > 1): stage streams
  // (stage 0 runs on the caller's stream; created on first use), the events
  // that order the stages (pready: level j's factors of the update in a slot
  // are assembled; pfree: the slot's update is through its top level) and
  // fork / join events.  pipeline = false keeps every batch sequential.
  bool pipeline = true;
  int pipe_nstages = 0;
  hipStream_t pstream[lv::kPipeStreams] = {};
  hipEvent_t pready[lv::kMaxLevel][lv::kMaxPipeSlots] = {};
  hipEvent_t pfree[lv::kMaxPipeSlots] = {};
  hipEvent_t pfork = nullptr;
  hipEvent_t pjoin[lv::kPipeStreams] = {};

  // stored powers held outside the workspace (set by the allocation-free
  // update entry point; null for views created on a workspace)
  char* pext[lv::kMaxLevel + 1] = {};
  template <typename T> T* P(int j) const { return reinterpret_cast<T*>(pext[j] ? pext[j] : base + L.P[j]); }
  template <typename T> T* slabU() const { return reinterpret_cast<T*>(base + L.slabU); }
  template <typename T> T* slabV() const { return reinterpret_cast<T*>(base + L.slabV); }
  template <typename T> T* slabU(int slot) const { return reinterpret_cast<T*>(base + L.pslabU[slot]); }
  template <typename T> T* slabV(int slot) const { return reinterpret_cast<T*>(base + L.pslabV[slot]); }
  template <typename T> T* partX(int j) const { return reinterpret_cast<T*>(base + L.partX[j]); }
  template <typename T> T* partY(int j) const { return reinterpret_cast<T*>(base + L.partY[j]); }
  double* partG(int j) const { return reinterpret_cast<double*>(base + L.partG[j]); }
  template <typename T> T* S(int j) const { return reinterpret_cast<T*>(base + L.S[j]); }
  template <typename T> T* slabQ() const { return reinterpret_cast<T*>(base + L.slabQ); }
  template <typename T> T* slabW() const { return reinterpret_cast<T*>(base + L.slabW); }
  template <typename T> T* partXs(int j) const { return reinterpret_cast<T*>(base + L.partXs[j]); }
  template <typename T> T* partYs(int j) const { return reinterpret_cast<T*>(base + L.partYs[j]); }
  double* partGs(int j) const { return reinterpret_cast<double*>(base + L.partGs[j]); }
  double* sscratch(int i) const { return reinterpret_cast<double*>(base + L.sscratch[i]); }
  template <typename T> T* Tg(int j) const { return reinterpret_cast<T*>(base + L.T[j]); }
  template <typename T> T* T0() const { return reinterpret_cast<T*>(base + L.T0); }
  template <typename T> T* Bg() const { return reinterpret_cast<T*>(base + L.B); }
  template <typename T> T* D(int i) const { return reinterpret_cast<T*>(base + L.D[i]); }
  template <typename T> T* partXT() const { return reinterpret_cast<T*>(base + L.partXT); }
  template <typename T> T* partYT() const { return reinterpret_cast<T*>(base + L.partYT); }
  double* atbA() const { return reinterpret_cast<double*>(base + L.atbA); }
  double* atbG() const { return reinterpret_cast<double*>(base + L.atbG); }
  template <typename T> T* Yf(int j) const { return reinterpret_cast<T*>(base + L.Y[j]); }
  template <typename T> T* Ztf(int j) const { return reinterpret_cast<T*>(base + L.Zt[j]); }
  // skip-model T_{(q+1)s}, its Y and Z^T slabs (q = 1 .. nsk)
  template <typename T> T* Tskp(int q) const { return reinterpret_cast<T*>(base + L.Tsk + (size_t)(q - 1) * L.tstride); }
  template <typename T> T* Yskp(int q) const { return reinterpret_cast<T*>(base + L.Ysk + (size_t)(q - 1) * L.ystride); }
  template <typename T> T* Ztskp(int q) const { return reinterpret_cast<T*>(base + L.Ztsk + (size_t)(q - 1) * L.zstride); }
  double* atbB() const { return reinterpret_cast<double*>(base + L.atbB); }
  double* gT(int i) const { return reinterpret_cast<double*>(base + L.gT[i]); }
  double* gTmp() const { return reinterpret_cast<double*>(base + L.gTmp); }
  double* gB() const { return reinterpret_cast<double*>(base + L.gB); }
  uint16_t* shadow(int j) const { return reinterpret_cast<uint16_t*>(base + L.shadow[j]); }
  bool shadowed() const { return mode == LV_FP32_BF16SHADOW; }
  double* scratch(int i) const { return reinterpret_cast<double*>(base + L.scratch[i]); }
  double* zpad() const { return reinterpret_cast<double*>(base + L.probe); }
  double* drift_z() const { return reinterpret_cast<double*>(base + L.drift_z); }
  double* Pz(int j) const { return zpad() + (size_t)(1 + j) * L.n_pad; }
  double* PPz(int j) const { return zpad() + (size_t)(L.m + 2 + j) * L.n_pad; }
  double* residuals() const { return zpad() + (size_t)(2 * L.m + 2) * L.n_pad; }
  int* gate() const { return reinterpret_cast<int*>(residuals() + lv::kMaxLevel); }
  unsigned long long* drift_counter() const {
    return reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(residuals() + lv::kMaxLevel) + 64);
  }
};
