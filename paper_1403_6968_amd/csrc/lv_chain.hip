// Matrix-power views under the linear, skip-s and exponential iterative
// models (Sec. 3.2, Table 1), maintained by IncrLin / IncrSkip-s / IncrExp
// (App. A).  Every stored P_c is a product P_a P_b of two earlier stored
// matrices (linear: a = 1, b = c - 1; skip-s: a = s, b = c - s beyond s;
// exponential: a = b = c/2), and its delta is factored as
//     U_c = [U_a, P_a U_b + U_a (V_a^T U_b)],   V_c = [P_b^T V_a, V_b]
// from the OLD matrices; then every stored matrix takes P_c += U_c V_c^T.
// Each stored matrix has its own factor slabs (width c * r_pad padded to a
// power of two): in the linear and skip models U_b is transformed, not
// extended, so the prefix layout of the exponential view does not apply.
#include "linview.h"
#include "lv_internal.h"
#include "lv_view_impl.h"

#include <new>
#include <utility>
#include <vector>

using namespace lv;

namespace lv {
namespace {

constexpr int kMaxChainWidth = 128;   // k * r_pad (the read-only passes take up to 128 columns)
constexpr int kMaxChainStored = 128;

// One thread per (row, column) of the new slabs, column < Wc:
//   col < wa:           U_c = U_a,                 V_c = sum_t partY[t]  (P_b^T V_a)
//   wa <= col < wa+wb:  U_c = sum_t partX[t] + U_a G  (P_a U_b + U_a (V_a^T U_b)),  V_c = V_b
//   otherwise zero.  Partial sums in tile order, double accumulation.
template <typename T>
__global__ void __launch_bounds__(256)
k_chain_tail(const T* __restrict__ partX, int nct, const T* __restrict__ partY, int nrt, const double* __restrict__ G,
             const T* __restrict__ Ua, int Wa, int wa, const T* __restrict__ Vb, int Wb, int wb,
             T* __restrict__ Uc, T* __restrict__ Vc, int Wc, int64_t n_pad) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n_pad * Wc) return;
  const int64_t row = idx / Wc;
  const int col = (int)(idx % Wc);
  double u = 0.0, v = 0.0;
  if (col < wa) {
    u = (double)Ua[row * Wa + col];
    for (int t = 0; t < nrt; ++t) v += (double)partY[((int64_t)t * n_pad + row) * Wa + col];
  } else if (col < wa + wb) {
    const int j = col - wa;
    for (int t = 0; t < nct; ++t) u += (double)partX[((int64_t)t * n_pad + row) * Wb + j];
    for (int d = 0; d < wa; ++d) u = fma((double)Ua[row * Wa + d], G[d * Wb + j], u);
    v = (double)Vb[row * Wb + j];
  }
  Uc[idx] = (T)u;
  Vc[idx] = (T)v;
}

}  // namespace
}  // namespace lv

struct lv_chain {
  int64_t n, n_pad;
  int k, s, model, r_max, r_pad, elem, nct, nrt;
  lv_mode mode;
  std::vector<int> pw;       // stored powers, pw[0] = 1
  std::vector<int> Wd;       // padded slab width of each stored matrix
  struct Step { int c, a, b; };
  std::vector<Step> steps;   // products in evaluation order (indices into pw)
  std::vector<size_t> P, sU, sV;
  size_t partX = 0, partY = 0, partXd = 0, partG = 0, d64[3] = {};
  size_t total = 0;
  char* base = nullptr;
  int64_t updates = 0;

  template <typename T> T* Pm(int i) const { return reinterpret_cast<T*>(base + P[i]); }
  template <typename T> T* U(int i) const { return reinterpret_cast<T*>(base + sU[i]); }
  template <typename T> T* V(int i) const { return reinterpret_cast<T*>(base + sV[i]); }
  template <typename T> T* pX() const { return reinterpret_cast<T*>(base + partX); }
  template <typename T> T* pY() const { return reinterpret_cast<T*>(base + partY); }
  template <typename T> T* pXd() const { return reinterpret_cast<T*>(base + partXd); }
  double* pG() const { return reinterpret_cast<double*>(base + partG); }
  double* d(int i) const { return reinterpret_cast<double*>(base + d64[i]); }
};

namespace {

// Stored powers and products of a model (Table 1, matrix-powers column).
lv_status plan_chain(lv_chain& c) {
  std::vector<std::pair<int, int>> prods;   // (c, a) with b the previous product
  if (c.model == LV_MODEL_LIN) {
    for (int i = 2; i <= c.k; ++i) prods.push_back({i, 1});
  } else if (c.model == LV_MODEL_EXP) {
    for (int i = 2; i <= c.k; i *= 2) prods.push_back({i, i / 2});
  } else {
    for (int i = 2; i <= c.s; i *= 2) prods.push_back({i, i / 2});
    for (int i = 2 * c.s; i <= c.k; i += c.s) prods.push_back({i, c.s});
  }
  c.pw.assign(1, 1);
  for (auto& p : prods) c.pw.push_back(p.first);
  if ((int)c.pw.size() > kMaxChainStored) return fail(LV_EINVAL, "%d stored matrices exceed %d", (int)c.pw.size(), kMaxChainStored);
  auto index = [&](int power) {
    for (size_t i = 0; i < c.pw.size(); ++i) if (c.pw[i] == power) return (int)i;
    return -1;
  };
  c.steps.clear();
  for (size_t q = 0; q < prods.size(); ++q) {
    const int ci = (int)q + 1, ai = index(prods[q].second), bi = index(prods[q].first - prods[q].second);
    if (ai < 0 || bi != ci - 1) return fail(LV_EINVAL, "internal: product %d has no stored operands", prods[q].first);
    c.steps.push_back({ci, ai, bi});
  }
  return LV_OK;
}

lv_status check_chain(int64_t n, int k, int r_max, lv_mode mode, int model, int s) {
  if (mode != LV_FP64 && mode != LV_FP32) return fail(LV_EINVAL, "chain views take LV_FP64 or LV_FP32, got %d", (int)mode);
  if (n < 1 || n > kMaxOrder) return fail(LV_EINVAL, "n = %lld outside [1, %lld]", (long long)n, (long long)kMaxOrder);
  if (r_max < 1) return fail(LV_EINVAL, "r_max = %d < 1", r_max);
  if (k < 1) return fail(LV_EINVAL, "k = %d < 1", k);
  if (model == LV_MODEL_EXP) {
    if (!is_pow2(k)) return fail(LV_EINVAL, "the exponential model needs k a power of two, got %d", k);
  } else if (model == LV_MODEL_SKIP) {
    if (!is_pow2(s) || s > k || k % s != 0)
      return fail(LV_EINVAL, "the skip model needs s a power of two dividing k, got s = %d, k = %d", s, k);
  } else if (model != LV_MODEL_LIN) {
    return fail(LV_EINVAL, "unknown model %d", model);
  }
  if ((int64_t)k * next_pow2(r_max) > kMaxChainWidth)
    return fail(LV_EINVAL, "k * r_max (rounded up to a power of two) exceeds %d", kMaxChainWidth);
  return LV_OK;
}

lv_status layout_chain(lv_chain& c, int64_t n, int k, int r_max, lv_mode mode, int model, int s) {
  c.n = n; c.k = k; c.s = model == LV_MODEL_SKIP ? s : 0; c.model = model; c.r_max = r_max; c.mode = mode;
  c.r_pad = (int)next_pow2(r_max);
  c.elem = mode == LV_FP64 ? 8 : 4;
  c.n_pad = round_up(n, kPadOrder);
  c.nct = (int)(c.n_pad / tile_cols_bytes(c.elem));
  c.nrt = (int)((c.n_pad + kTileRows - 1) / kTileRows);
  lv_status st = plan_chain(c);
  if (st != LV_OK) return st;
  const int ns = (int)c.pw.size();
  c.Wd.resize(ns);
  int maxW = 1;
  for (int i = 0; i < ns; ++i) { c.Wd[i] = (int)next_pow2((int64_t)c.pw[i] * c.r_pad); maxW = c.Wd[i] > maxW ? c.Wd[i] : maxW; }
  size_t maxG = 1;
  for (auto& q : c.steps) { const size_t g = (size_t)c.Wd[q.a] * c.Wd[q.b]; maxG = g > maxG ? g : maxG; }
  size_t off = 0;
  const size_t mat = (size_t)c.n_pad * c.n_pad * c.elem;
  c.P.resize(ns); c.sU.resize(ns); c.sV.resize(ns);
  for (int i = 0; i < ns; ++i) { c.P[i] = off; off = align_up(off + mat); }
  for (int i = 0; i < ns; ++i) {
    const size_t slab = (size_t)c.n_pad * c.Wd[i] * c.elem;
    c.sU[i] = off; off = align_up(off + slab);
    c.sV[i] = off; off = align_up(off + slab);
  }
  c.partX = off; off = align_up(off + (size_t)c.nct * c.n_pad * maxW * c.elem);
  c.partXd = off; off = align_up(off + (size_t)c.nct * c.n_pad * maxW * c.elem);
  c.partY = off; off = align_up(off + (size_t)c.nrt * c.n_pad * maxW * c.elem);
  c.partG = off; off = align_up(off + (size_t)(c.n_pad / kAtbRows) * maxG * sizeof(double));
  if (mode == LV_FP32 && ns > 1)
    for (int i = 0; i < 3; ++i) { c.d64[i] = off; off = align_up(off + (size_t)c.n_pad * c.n_pad * sizeof(double)); }
  c.total = off;
  return LV_OK;
}

// Creation: the model's products in double precision (float views keep the
// running product and the fixed left operand in double and round each
// stored matrix once).
template <typename T>
lv_status build_chain_model(lv_chain* c, hipStream_t s) {
  const int64_t np = c->n_pad;
  if constexpr (sizeof(T) == 8) {
    for (auto& q : c->steps) {
      lv_status st = hip_check(launch_gemm<double>(c->Pm<double>(q.a), np, c->Pm<double>(q.b), np, c->Pm<double>(q.c),
                                                   np, np, s), "gemm f64");
      if (st != LV_OK) return st;
    }
    return LV_OK;
  } else {
    if (c->steps.empty()) return LV_OK;
    double* prev = c->d(0);
    double* next = c->d(1);
    double* mult = c->d(2);
    const int mult_pw = c->model == LV_MODEL_LIN ? 1 : c->model == LV_MODEL_SKIP ? c->s : -1;
    lv_status st = hip_check(launch_copy_pad<float, double>(c->Pm<float>(0), np, np, prev, np, np, s), "widen A");
    const size_t dbytes = (size_t)np * np * sizeof(double);
    if (st == LV_OK && mult_pw == 1)
      st = hip_check(hipMemcpyAsync(mult, prev, dbytes, hipMemcpyDeviceToDevice, s), "keep A");
    for (auto& q : c->steps) {
      if (st != LV_OK) return st;
      const double* lhs = q.a == q.b ? prev : mult;
      st = hip_check(launch_gemm<double>(lhs, np, prev, np, next, np, np, s), "gemm f64");
      if (st == LV_OK)
        st = hip_check(launch_copy_pad<double, float>(next, np, np, c->Pm<float>(q.c), np, np, s), "round P");
      std::swap(prev, next);
      if (st == LV_OK && c->pw[q.c] == mult_pw && mult_pw != 1)
        st = hip_check(hipMemcpyAsync(mult, prev, dbytes, hipMemcpyDeviceToDevice, s), "keep P_s");
    }
    return st;
  }
}

// Read-only products of one step: X = P_a U_b (column-tile partials, width
// W_b) and Y = P_b^T V_a (row-tile partials, width W_a).  One pass when
// a = b; otherwise one pass over each matrix (the unused product of each
// pass goes to a discard buffer on the vector path; the float matrix-core
// pass from width 16 computes only what is asked).
template <typename T>
lv_status step_products(lv_chain* c, const lv_chain::Step& q, hipStream_t s) {
  const int64_t np = c->n_pad;
  const int Wa = c->Wd[q.a], Wb = c->Wd[q.b];
  const T* Ub = c->U<T>(q.b);
  const T* Va = c->V<T>(q.a);
  auto pass = [&](const T* P, int R, const T* op1, const T* op2, T* px, T* py, int want) -> hipError_t {
    if (skinny_on_mfma(R, (int)sizeof(T)))
      return launch_skinny_f32(R, reinterpret_cast<const float*>(P), np, np, kTileRows,
                               reinterpret_cast<const float*>(op1), reinterpret_cast<const float*>(op2), R,
                               reinterpret_cast<float*>(px), reinterpret_cast<float*>(py), s, want);
    return launch_level_readonly<T>(R, P, np, np, kTileRows, op1, op2, R, px, py, s);
  };
  if (q.a == q.b)
    return hip_check(pass(c->Pm<T>(q.a), Wa, Ub, Va, c->pX<T>(), c->pY<T>(), kWantX | kWantY), "P U, P^T V");
  lv_status st = hip_check(pass(c->Pm<T>(q.a), Wb, Ub, Ub, c->pX<T>(), c->pY<T>(), kWantX), "P_a U_b");
  if (st != LV_OK) return st;
  return hip_check(pass(c->Pm<T>(q.b), Wa, Va, Va, c->pXd<T>(), c->pY<T>(), kWantY), "P_b^T V_a");
}

template <typename T>
lv_status chain_update(lv_chain* c, const T* U, const T* V, int r, int64_t ldu, int64_t ldv, hipStream_t s) {
  const int64_t np = c->n_pad;
  lv_status st = hip_check(launch_prep<T>(U, ldu, V, ldv, c->n, r, c->r_pad, c->U<T>(0), c->V<T>(0), c->r_pad, np, s),
                           "prep");
  for (auto& q : c->steps) {
    if (st != LV_OK) return st;
    const int Wa = c->Wd[q.a], Wb = c->Wd[q.b], Wc = c->Wd[q.c];
    st = step_products<T>(c, q, s);
    if (st == LV_OK)
      st = hip_check(launch_atb<T>(Wa, Wb, c->V<T>(q.a), Wa, c->U<T>(q.b), Wb, np, c->pG(), s), "V_a^T U_b");
    if (st == LV_OK) {
      hipLaunchKernelGGL((k_chain_tail<T>), dim3((unsigned)((np * Wc + 255) / 256)), dim3(256), 0, s, c->pX<T>(),
                         c->nct, c->pY<T>(), c->nrt, c->pG(), c->U<T>(q.a), Wa, c->pw[q.a] * c->r_pad, c->V<T>(q.b),
                         Wb, c->pw[q.b] * c->r_pad, c->U<T>(q.c), c->V<T>(q.c), Wc, np);
      st = hip_check(hipGetLastError(), "chain tail");
    }
  }
  for (size_t i = 0; i < c->pw.size() && st == LV_OK; ++i)
    st = hip_check(launch_level_update<T>(c->Wd[i], c->Pm<T>((int)i), np, np, c->U<T>((int)i), c->V<T>((int)i),
                                          c->Wd[i], s), "P += U V^T");
  return st;
}

}  // namespace

extern "C" {

size_t lv_chain_footprint(int64_t n, int k, int r_max, lv_mode mode, int model, int s) {
  if (check_chain(n, k, r_max, mode, model, s) != LV_OK) return 0;
  lv_chain c;
  if (layout_chain(c, n, k, r_max, mode, model, s) != LV_OK) return 0;
  return c.total;
}

lv_status lv_chain_create(const void* A, int64_t n, int64_t lda, int k, int r_max, lv_mode mode, int model, int s,
                          void* workspace, size_t ws_bytes, void* stream, lv_chain** out) {
  g_err[0] = 0;
  if (!out) return fail(LV_EINVAL, "out is NULL");
  *out = nullptr;
  lv_status st = check_chain(n, k, r_max, mode, model, s);
  if (st != LV_OK) return st;
  if (!A || !workspace) return fail(LV_EINVAL, "A or workspace is NULL");
  if (lda < n) return fail(LV_EINVAL, "lda = %lld < n = %lld", (long long)lda, (long long)n);
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(LV_ENOMEM, "workspace is not %zu-byte aligned", kAlign);
  lv_chain* c = new (std::nothrow) lv_chain();
  if (!c) return fail(LV_ENOMEM, "host allocation of the chain handle failed");
  st = layout_chain(*c, n, k, r_max, mode, model, s);
  if (st == LV_OK && ws_bytes < c->total) st = fail(LV_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, c->total);
  if (st != LV_OK) { delete c; return st; }
  c->base = static_cast<char*>(workspace);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  if (mode == LV_FP64) {
    st = hip_check(launch_copy_pad<double, double>(static_cast<const double*>(A), lda, n, c->Pm<double>(0), c->n_pad,
                                                   c->n_pad, hs), "copy A");
    if (st == LV_OK) st = build_chain_model<double>(c, hs);
  } else {
    st = hip_check(launch_copy_pad<float, float>(static_cast<const float*>(A), lda, n, c->Pm<float>(0), c->n_pad,
                                                 c->n_pad, hs), "copy A");
    if (st == LV_OK) st = build_chain_model<float>(c, hs);
  }
  if (st != LV_OK) { delete c; return st; }
  *out = c;
  return LV_OK;
}

lv_status lv_chain_update(lv_chain* c, const void* U, const void* V, int64_t r, int64_t ldu, int64_t ldv,
                          void* stream) {
  g_err[0] = 0;
  if (!c) return fail(LV_EINVAL, "chain is NULL");
  if (!U || !V) return fail(LV_EINVAL, "U or V is NULL");
  if (r < 1 || r > c->r_max) return fail(LV_EINVAL, "rank r = %lld outside [1, %d]", (long long)r, c->r_max);
  if (ldu < r || ldv < r) return fail(LV_EINVAL, "ldu/ldv smaller than r");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const lv_status st =
      c->mode == LV_FP64
          ? chain_update<double>(c, static_cast<const double*>(U), static_cast<const double*>(V), (int)r, ldu, ldv, s)
          : chain_update<float>(c, static_cast<const float*>(U), static_cast<const float*>(V), (int)r, ldu, ldv, s);
  if (st == LV_OK) c->updates += 1;
  return st;
}

lv_status lv_chain_read(const lv_chain* c, int power, void* out, int64_t ldo, void* stream) {
  g_err[0] = 0;
  if (!c || !out) return fail(LV_EINVAL, "chain or out is NULL");
  if (ldo < c->n) return fail(LV_EINVAL, "ldo < n");
  for (size_t i = 0; i < c->pw.size(); ++i)
    if (c->pw[i] == power) {
      const size_t es = c->elem;
      return hip_check(hipMemcpy2DAsync(out, ldo * es, c->base + c->P[i], c->n_pad * es, c->n * es, c->n,
                                        hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)),
                       "read");
    }
  return fail(LV_EINVAL, "power %d is not stored by this model", power);
}

int lv_chain_powers(const lv_chain* c, int* powers, int cap) {
  if (!c) return -1;
  const int ns = (int)c->pw.size();
  for (int i = 0; i < ns && i < cap && powers; ++i) powers[i] = c->pw[i];
  return ns;
}

void lv_chain_destroy(lv_chain* c) { delete c; }

}  // extern "C"
