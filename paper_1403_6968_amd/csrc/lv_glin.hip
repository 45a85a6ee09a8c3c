// The general form T_{i+1} = A T_i + B under the linear model (Sec. 3.2,
// Table 1; App. B, linear model): every T_1 .. T_k is stored and kept
// current under Delta A = U V^T by one of the three strategies of Table 2:
//   re-evaluation  A += U V^T, then T_i = A T_{i-1} + B for i = 1 .. k;
//   hybrid         Delta T_1 = U (V^T T_0),
//                  Delta T_i = A Delta T_{i-1} + U (V^T (T_{i-1} + Delta T_{i-1}))
//                  (old A and T), each one dense n x p matrix;
//   incremental    Delta T_i = Y_i Z_i^T, Y_1 = U, Z_1 = T_0^T V,
//                  Y_i = [U, A Y_{i-1} + U (V^T Y_{i-1})], Z_i = [T_{i-1}^T V, Z_{i-1}]
//                  (old A and T; widths i r), then every T_i += Y_i Z_i^T;
// and A += U V^T after the hybrid and incremental steps.  Products with A
// run as read-only passes (width <= 128; from 16 on the float matrix cores)
// or, for wide operands (p > 64), on the MFMA GEMM.
#include "linview.h"
#include "lv_internal.h"
#include "lv_view_impl.h"

#include <new>

using namespace lv;

namespace lv {
namespace {

constexpr int kGlinMaxK = 256;
constexpr int kGlinNarrow = 64;      // p up to this: read-only passes (p padded to a power of two)
constexpr int kGlinMaxCols = 4096;   // wider p: padded to a multiple of 128, products on the MFMA GEMM
constexpr int kGlinMaxWidth = 128;   // k * r_pad for incremental evaluation

// One thread per (row, column) of an n_pad x pp result:
//   d = sum_t partX[t] + full + sum_c U[row][c] a[c][col]   (double)
// assign: Tio = d + B (re-evaluation); else Dout = d, Tio += d (hybrid).
template <typename T>
__global__ void __launch_bounds__(256)
k_glin_tail(const T* __restrict__ partX, int nct, const T* __restrict__ full, const T* __restrict__ U, int R,
            const double* __restrict__ a, const T* __restrict__ B, T* __restrict__ Dout, T* __restrict__ Tio,
            int64_t n_pad, int pp, int assign) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n_pad * pp) return;
  const int64_t row = idx / pp;
  const int col = (int)(idx % pp);
  const int64_t stride = n_pad * pp;
  double d = 0.0;
  for (int t = 0; t < nct; ++t) d += (double)partX[t * stride + idx];
  if (full != nullptr) d += (double)full[idx];
  for (int c = 0; c < R; ++c) d = fma((double)U[row * R + c], a[c * pp + col], d);
  if (assign) {
    Tio[idx] = (T)(d + (double)B[idx]);
  } else {
    Dout[idx] = (T)d;
    Tio[idx] = (T)((double)Tio[idx] + d);
  }
}

}  // namespace
}  // namespace lv

struct lv_glin {
  int64_t n, n_pad;
  int k, p, pp, r_max, r_pad, elem, nct, nrt, strategy, maxw;
  lv_mode mode;
  size_t A, Tb, Bb, D[2], sU, sV, partX, partY, full, atbA, atbG, Yb, Zb, A64, gT[2], gB, total;
  size_t Toff(int i) const { return Tb + (size_t)i * align_up((size_t)n_pad * pp * elem); }
  int wy(int i) const { return i * r_pad; }                         // width of Y_i, Z_i
  int WY(int i) const { return (int)next_pow2(wy(i)); }
  size_t Yoff(int i) const { return Yb + (size_t)(i - 2) * align_up((size_t)n_pad * maxw * elem); }   // i >= 2
  size_t Zoff(int i) const { return Zb + (size_t)(i - 1) * align_up((size_t)maxw * pp * elem); }
  char* base = nullptr;
  int64_t updates = 0;
  template <typename T> T* at(size_t off) const { return reinterpret_cast<T*>(base + off); }
  double* d64(size_t off) const { return reinterpret_cast<double*>(base + off); }
};

namespace {

lv_status check_glin(int64_t n, int k, int r_max, lv_mode mode, int64_t p, int strategy) {
  if (mode != LV_FP64 && mode != LV_FP32) return fail(LV_EINVAL, "linear-model views take LV_FP64 or LV_FP32");
  if (n < 1 || n > kMaxOrder) return fail(LV_EINVAL, "n = %lld outside [1, %lld]", (long long)n, (long long)kMaxOrder);
  if (k < 1 || k > kGlinMaxK) return fail(LV_EINVAL, "k = %d outside [1, %d]", k, kGlinMaxK);
  if (r_max < 1) return fail(LV_EINVAL, "r_max = %d < 1", r_max);
  if (p < 1 || p > kGlinMaxCols) return fail(LV_EINVAL, "p = %lld outside [1, %d]", (long long)p, kGlinMaxCols);
  if (strategy != LV_GLIN_REEVAL && strategy != LV_GLIN_HYBRID && strategy != LV_GLIN_INCR)
    return fail(LV_EINVAL, "unknown strategy %d", strategy);
  if (strategy == LV_GLIN_INCR && (int64_t)k * next_pow2(r_max) > kGlinMaxWidth)
    return fail(LV_EINVAL, "incremental evaluation needs k * r_max (rounded up to a power of two) <= %d", kGlinMaxWidth);
  return LV_OK;
}

void layout_glin(lv_glin& g, int64_t n, int k, int r_max, lv_mode mode, int64_t p, int strategy) {
  g.n = n; g.k = k; g.r_max = r_max; g.mode = mode; g.p = (int)p; g.strategy = strategy;
  g.elem = mode == LV_FP64 ? 8 : 4;
  g.n_pad = round_up(n, kPadOrder);
  g.r_pad = (int)next_pow2(r_max);
  g.pp = p <= kGlinNarrow ? (int)next_pow2(p) : (int)round_up(p, 128);
  g.nct = (int)(g.n_pad / tile_cols_bytes(g.elem));
  g.nrt = (int)((g.n_pad + kTileRows - 1) / kTileRows);
  g.maxw = strategy == LV_GLIN_INCR ? (int)next_pow2((int64_t)k * g.r_pad) : 1;
  const size_t e = g.elem, np = g.n_pad, pp = g.pp;
  const int xw = strategy == LV_GLIN_INCR ? g.maxw : (g.pp <= kGlinNarrow ? g.pp : 1);   // read-only pass width
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t at = off; off = align_up(off + bytes); return at; };
  g.A = take(np * np * e);
  g.Tb = off;
  for (int i = 0; i <= k; ++i) take(np * pp * e);      // T_0 .. T_k
  g.Bb = take(np * pp * e);
  g.sU = take(np * g.r_pad * e);
  g.sV = take(np * g.r_pad * e);
  g.partX = take((size_t)g.nct * np * xw * e);
  g.partY = take((size_t)g.nrt * np * xw * e);
  g.atbA = take((np / kAtbRows) * g.r_pad * pp * sizeof(double));
  g.D[0] = g.D[1] = g.full = g.atbG = g.Yb = g.Zb = 0;
  if (strategy == LV_GLIN_HYBRID) { g.D[0] = take(np * pp * e); g.D[1] = take(np * pp * e); }
  if (strategy != LV_GLIN_INCR && g.pp > kGlinNarrow) g.full = take(np * pp * e);
  if (strategy == LV_GLIN_INCR) {
    g.atbG = take((np / kAtbRows) * g.r_pad * g.maxw * sizeof(double));
    g.Yb = off;
    for (int i = 2; i <= k; ++i) take(np * g.maxw * e);
    g.Zb = off;
    for (int i = 1; i <= k; ++i) take((size_t)g.maxw * pp * e);
  }
  g.A64 = take(mode == LV_FP32 ? np * np * sizeof(double) : 0);
  g.gT[0] = take(np * pp * sizeof(double));
  g.gT[1] = take(np * pp * sizeof(double));
  g.gB = take(np * pp * sizeof(double));
  g.total = off;
}

// Creation: T_i = A T_{i-1} + B in double from the double A, each rounded once.
template <typename T>
lv_status glin_build(lv_glin* g, hipStream_t s) {
  const int64_t np = g->n_pad;
  const int pp = g->pp;
  const double* A64 = g->mode == LV_FP64 ? g->d64(g->A) : g->d64(g->A64);
  lv_status st = LV_OK;
  if (g->mode == LV_FP32)
    st = hip_check(launch_copy_pad<float, double>(g->at<float>(g->A), np, np, g->d64(g->A64), np, np, s), "widen A");
  if (st == LV_OK)
    st = hip_check(launch_copy_rect<T, double>(g->at<T>(g->Toff(0)), pp, np, pp, g->d64(g->gT[0]), np, pp, s), "T_0");
  if (st == LV_OK)
    st = hip_check(launch_copy_rect<T, double>(g->at<T>(g->Bb), pp, np, pp, g->d64(g->gB), np, pp, s), "B");
  for (int i = 1; i <= g->k && st == LV_OK; ++i) {
    double* prev = g->d64(g->gT[(i - 1) & 1]);
    double* next = g->d64(g->gT[i & 1]);
    if (pp <= kGlinNarrow) {
      st = hip_check(launch_gemm_np(pp, A64, np, prev, next, g->d64(g->gB), np, s), "A T + B");
    } else {
      st = hip_check(launch_gemm_rect<double>(A64, np, prev, pp, next, pp, np, pp, np, s), "A T");
      if (st == LV_OK) st = hip_check(launch_add<double>(next, g->d64(g->gB), np * pp, s), "+ B");
    }
    if (st == LV_OK)
      st = hip_check(launch_copy_rect<double, T>(next, pp, np, pp, g->at<T>(g->Toff(i)), np, pp, s), "round T");
  }
  return st;
}

// out = A M (M n_pad x w, row stride sm) with the OLD A: partials of a
// read-only pass (w <= 128) or, for wide M (w > 64, a multiple of 128), the
// full product on the MFMA GEMM.  Returns the partial count (0 for the full
// product, which goes to `full`).
template <typename T>
lv_status glin_amul(lv_glin* g, const T* M, int w, int sm, hipStream_t s, int* nct_out) {
  const int64_t np = g->n_pad;
  if (w > kGlinNarrow && g->full != 0) {
    *nct_out = 0;
    return hip_check(launch_gemm_rect<T>(g->at<T>(g->A), np, M, sm, g->at<T>(g->full), g->pp, np, w, np, s), "A M");
  }
  *nct_out = g->nct;
  if (skinny_on_mfma(w, (int)sizeof(T)))
    return hip_check(launch_skinny_f32(w, reinterpret_cast<const float*>(g->at<T>(g->A)), np, np, kTileRows,
                                       reinterpret_cast<const float*>(M), reinterpret_cast<const float*>(M), sm,
                                       g->at<float>(g->partX), g->at<float>(g->partY), s, kWantX),
                     "A M");
  return hip_check(launch_level_readonly<T>(w, g->at<T>(g->A), np, np, kTileRows, M, M, sm, g->at<T>(g->partX),
                                            g->at<T>(g->partY), s),
                   "A M");
}

// The product of glin_amul enters as `nct` partials, or as the full
// product when with_product is set and nct is 0; with_product = false: no
// product term at all (the first hybrid step).
template <typename T>
lv_status glin_tail(lv_glin* g, bool with_product, int nct, int R, const double* a, bool assign, T* Dout, T* Tio,
                    hipStream_t s) {
  const int64_t np = g->n_pad;
  const T* full = with_product && nct == 0 ? g->at<T>(g->full) : nullptr;
  hipLaunchKernelGGL((k_glin_tail<T>), dim3((unsigned)((np * g->pp + 255) / 256)), dim3(256), 0, s,
                     g->at<T>(g->partX), with_product ? nct : 0, full, g->at<T>(g->sU), R, a, g->at<T>(g->Bb), Dout,
                     Tio, np, g->pp, assign ? 1 : 0);
  return hip_check(hipGetLastError(), "tail");
}

template <typename T>
lv_status glin_update(lv_glin* g, const T* U, const T* V, int r, int64_t ldu, int64_t ldv, hipStream_t s) {
  const int64_t np = g->n_pad;
  const int R = g->r_pad, pp = g->pp;
  T* sU = g->at<T>(g->sU);
  T* sV = g->at<T>(g->sV);
  lv_status st = hip_check(launch_prep<T>(U, ldu, V, ldv, g->n, r, R, sU, sV, R, np, s), "prep");
  if (st != LV_OK) return st;
  auto update_A = [&]() {
    return hip_check(launch_level_update<T>(R, g->at<T>(g->A), np, np, sU, sV, R, s), "A += U V^T");
  };
  int nct = 0;
  if (g->strategy == LV_GLIN_REEVAL) {
    st = update_A();
    for (int i = 1; i <= g->k && st == LV_OK; ++i) {
      st = glin_amul<T>(g, g->at<T>(g->Toff(i - 1)), pp, pp, s, &nct);
      if (st == LV_OK) st = glin_tail<T>(g, true, nct, 0, nullptr, true, nullptr, g->at<T>(g->Toff(i)), s);
    }
    return st;
  }
  if (g->strategy == LV_GLIN_HYBRID) {
    // D_1 = U (V^T T_0), T_1 += D_1
    st = hip_check(launch_atb<T>(R, pp, sV, R, g->at<T>(g->Toff(0)), pp, np, g->d64(g->atbA), s), "V^T T_0");
    if (st == LV_OK)
      st = glin_tail<T>(g, false, 0, R, g->d64(g->atbA), false, g->at<T>(g->D[0]), g->at<T>(g->Toff(1)), s);
    for (int i = 2; i <= g->k && st == LV_OK; ++i) {
      // D_i = A D_{i-1} + U (V^T T_{i-1}), T_{i-1} already holding T + D
      st = glin_amul<T>(g, g->at<T>(g->D[i & 1]), pp, pp, s, &nct);
      if (st == LV_OK)
        st = hip_check(launch_atb<T>(R, pp, sV, R, g->at<T>(g->Toff(i - 1)), pp, np, g->d64(g->atbA), s), "V^T T");
      if (st == LV_OK)
        st = glin_tail<T>(g, true, nct, R, g->d64(g->atbA), false, g->at<T>(g->D[(i - 1) & 1]), g->at<T>(g->Toff(i)),
                          s);
    }
    return st == LV_OK ? update_A() : st;
  }
  // incremental: Z_1^T = V^T T_0, Y_1 = U; then Y_i, Z_i; then every T_i += Y_i Z_i^T
  st = hip_check(launch_atb<T>(R, pp, sV, R, g->at<T>(g->Toff(0)), pp, np, g->d64(g->atbA), s), "V^T T_0");
  if (st == LV_OK)
    st = hip_check(launch_gfac_z<T>(g->d64(g->atbA), nullptr, 0, nullptr, R, g->at<T>(g->Zoff(1)), g->WY(1), pp, s),
                   "Z_1");
  for (int i = 2; i <= g->k && st == LV_OK; ++i) {
    const T* Yp = i == 2 ? sU : g->at<T>(g->Yoff(i - 1));
    const int sp = i == 2 ? R : g->WY(i - 1);
    st = glin_amul<T>(g, Yp, g->WY(i - 1), sp, s, &nct);
    if (st == LV_OK)
      st = hip_check(launch_atb<T>(R, g->WY(i - 1), sV, R, Yp, sp, np, g->d64(g->atbG), s), "V^T Y");
    if (st == LV_OK)
      st = hip_check(launch_atb<T>(R, pp, sV, R, g->at<T>(g->Toff(i - 1)), pp, np, g->d64(g->atbA), s), "V^T T");
    if (st == LV_OK)
      st = hip_check(launch_gfac_y<T>(g->at<T>(g->partX), nct, g->WY(i - 1), sU, nullptr, R, R, g->d64(g->atbG),
                                      g->WY(i - 1), g->wy(i - 1), g->at<T>(g->Yoff(i)), g->WY(i), np, s),
                     "Y");
    if (st == LV_OK)
      st = hip_check(launch_gfac_z<T>(g->d64(g->atbA), g->at<T>(g->Zoff(i - 1)), g->wy(i - 1), nullptr, R,
                                      g->at<T>(g->Zoff(i)), g->WY(i), pp, s),
                     "Z");
  }
  for (int i = 1; i <= g->k && st == LV_OK; ++i)
    st = hip_check(launch_rank_rect<T>(g->at<T>(g->Toff(i)), i == 1 ? sU : g->at<T>(g->Yoff(i)), i == 1 ? R : g->WY(i),
                                       g->at<T>(g->Zoff(i)), g->wy(i), np, pp, s),
                   "T += Y Z^T");
  return st == LV_OK ? update_A() : st;
}

}  // namespace

extern "C" {

size_t lv_glin_footprint(int64_t n, int k, int r_max, lv_mode mode, int64_t p, int strategy) {
  if (check_glin(n, k, r_max, mode, p, strategy) != LV_OK) return 0;
  lv_glin g;
  layout_glin(g, n, k, r_max, mode, p, strategy);
  return g.total;
}

lv_status lv_glin_create(const void* A, int64_t n, int64_t lda, int k, int r_max, lv_mode mode, const void* T0,
                         int64_t ldt, const void* B, int64_t ldb, int64_t p, int strategy, void* workspace,
                         size_t ws_bytes, void* stream, lv_glin** out) {
  g_err[0] = 0;
  if (!out) return fail(LV_EINVAL, "out is NULL");
  *out = nullptr;
  lv_status st = check_glin(n, k, r_max, mode, p, strategy);
  if (st != LV_OK) return st;
  if (!A || !T0 || !B || !workspace) return fail(LV_EINVAL, "A, T0, B or workspace is NULL");
  if (lda < n || ldt < p || ldb < p) return fail(LV_EINVAL, "lda < n, ldt < p or ldb < p");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(LV_ENOMEM, "workspace is not %zu-byte aligned", kAlign);
  lv_glin* g = new (std::nothrow) lv_glin();
  if (!g) return fail(LV_ENOMEM, "host allocation of the handle failed");
  layout_glin(*g, n, k, r_max, mode, p, strategy);
  if (ws_bytes < g->total) {
    const size_t need = g->total;
    delete g;
    return fail(LV_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  }
  g->base = static_cast<char*>(workspace);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t np = g->n_pad;
  if (mode == LV_FP64) {
    st = hip_check(launch_copy_pad<double, double>(static_cast<const double*>(A), lda, n, g->at<double>(g->A), np, np, s),
                   "copy A");
    if (st == LV_OK)
      st = hip_check(launch_copy_rect<double, double>(static_cast<const double*>(T0), ldt, n, (int)p,
                                                      g->at<double>(g->Toff(0)), np, g->pp, s), "copy T_0");
    if (st == LV_OK)
      st = hip_check(launch_copy_rect<double, double>(static_cast<const double*>(B), ldb, n, (int)p, g->at<double>(g->Bb),
                                                      np, g->pp, s), "copy B");
    if (st == LV_OK) st = glin_build<double>(g, s);
  } else {
    st = hip_check(launch_copy_pad<float, float>(static_cast<const float*>(A), lda, n, g->at<float>(g->A), np, np, s),
                   "copy A");
    if (st == LV_OK)
      st = hip_check(launch_copy_rect<float, float>(static_cast<const float*>(T0), ldt, n, (int)p,
                                                    g->at<float>(g->Toff(0)), np, g->pp, s), "copy T_0");
    if (st == LV_OK)
      st = hip_check(launch_copy_rect<float, float>(static_cast<const float*>(B), ldb, n, (int)p, g->at<float>(g->Bb),
                                                    np, g->pp, s), "copy B");
    if (st == LV_OK) st = glin_build<float>(g, s);
  }
  if (st != LV_OK) { delete g; return st; }
  *out = g;
  return LV_OK;
}

lv_status lv_glin_update(lv_glin* g, const void* U, const void* V, int64_t r, int64_t ldu, int64_t ldv, void* stream) {
  g_err[0] = 0;
  if (!g || !U || !V) return fail(LV_EINVAL, "handle, U or V is NULL");
  if (r < 1 || r > g->r_max) return fail(LV_EINVAL, "rank r = %lld outside [1, %d]", (long long)r, g->r_max);
  if (ldu < r || ldv < r) return fail(LV_EINVAL, "ldu/ldv smaller than r");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const lv_status st =
      g->mode == LV_FP64
          ? glin_update<double>(g, static_cast<const double*>(U), static_cast<const double*>(V), (int)r, ldu, ldv, s)
          : glin_update<float>(g, static_cast<const float*>(U), static_cast<const float*>(V), (int)r, ldu, ldv, s);
  if (st == LV_OK) g->updates += 1;
  return st;
}

lv_status lv_glin_read(const lv_glin* g, int i, void* out, int64_t ldo, void* stream) {
  g_err[0] = 0;
  if (!g || !out) return fail(LV_EINVAL, "handle or out is NULL");
  if (i < 0 || i > g->k) return fail(LV_EINVAL, "T_%d is not stored (0 <= i <= %d)", i, g->k);
  if (ldo < g->p) return fail(LV_EINVAL, "ldo < p");
  const size_t es = g->elem;
  return hip_check(hipMemcpy2DAsync(out, ldo * es, g->base + g->Toff(i), g->pp * es, g->p * es, g->n,
                                    hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)),
                   "read");
}

void lv_glin_destroy(lv_glin* g) { delete g; }

}  // extern "C"
