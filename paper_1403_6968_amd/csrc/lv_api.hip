// C ABI of liblinview: argument validation, workspace layout, and the order
// of kernel launches for view creation, updates, re-anchoring and the
// re-evaluation baseline.
#include "linview.h"
#include "lv_internal.h"

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "lv_view_impl.h"

using namespace lv;

namespace lv {
thread_local char g_err[512] = "";

lv_status fail(lv_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}
}  // namespace lv

namespace {

// Stored powers P_1..P_m from P_0 by repeated squaring in double precision
// (Table 1, exponential model), then one rounding to the storage type.
// With a non-null gate every kernel of the chain runs only if *gate != 0.
// General form, creation step of level j in double (Table 1, exponential
// model): T_1 = A T_0 + B for j = 0, else T_{2^j} = P T_{2^(j-1)} + S B with
// P, S the double P_{j-1}, S_{j-1}; the double T ping-pongs in gT, the
// stored T_{2^j} is its rounding.
template <typename T>
lv_status general_step(lv_view* v, int j, const double* P, const double* S, int64_t ld, hipStream_t s,
                       const int* gate) {
  const Layout& L = v->L;
  lv_status st = LV_OK;
  if (j == 0) {
    st = hip_check(launch_copy_rect<T, double>(v->T0<T>(), L.pp, L.n_pad, L.pp, v->gT(0), L.n_pad, L.pp, s, gate),
                   "widen T_0");
    if (st == LV_OK)
      st = hip_check(launch_copy_rect<T, double>(v->Bg<T>(), L.pp, L.n_pad, L.pp, v->gB(), L.n_pad, L.pp, s, gate),
                     "widen B");
    if (st == LV_OK && L.gfac) {
      st = hip_check(launch_gemm_rect<double>(P, ld, v->gT(0), L.pp, v->gT(1), L.pp, L.n_pad, L.pp, L.n_pad, s, gate),
                     "A T_0");
      if (st == LV_OK) st = hip_check(launch_add<double>(v->gT(1), v->gB(), L.n_pad * L.pp, s, gate), "+ B");
    } else if (st == LV_OK) {
      st = hip_check(launch_gemm_np(L.pp, P, ld, v->gT(0), v->gT(1), v->gB(), L.n_pad, s, gate), "T_1 = A T_0 + B");
    }
  } else if (L.gfac) {
    st = hip_check(launch_gemm_rect<double>(S, ld, v->gB(), L.pp, v->gTmp(), L.pp, L.n_pad, L.pp, L.n_pad, s, gate),
                   "S B");
    if (st == LV_OK)
      st = hip_check(launch_gemm_rect<double>(P, ld, v->gT(j & 1), L.pp, v->gT((j + 1) & 1), L.pp, L.n_pad, L.pp,
                                              L.n_pad, s, gate),
                     "P T");
    if (st == LV_OK) st = hip_check(launch_add<double>(v->gT((j + 1) & 1), v->gTmp(), L.n_pad * L.pp, s, gate), "+ S B");
  } else {
    st = hip_check(launch_gemm_np(L.pp, S, ld, v->gB(), v->gTmp(), nullptr, L.n_pad, s, gate), "S B");
    if (st == LV_OK)
      st = hip_check(launch_gemm_np(L.pp, P, ld, v->gT(j & 1), v->gT((j + 1) & 1), v->gTmp(), L.n_pad, s, gate),
                     "T = P T + S B");
  }
  if (st == LV_OK)
    st = hip_check(launch_copy_rect<double, T>(v->gT((j + 1) & 1), L.pp, L.n_pad, L.pp, v->Tg<T>(j), L.n_pad, L.pp,
                                                s, gate),
                   "round T");
  return st;
}

// Skip model, creation: T_{(q+1)s} = P_s T_{qs} + S_s B for q = 1 .. nsk in
// double from the double P_s, S_s (the last level's T_s sits in gT((m+1) & 1)).
template <typename T>
lv_status skip_steps(lv_view* v, const double* P, const double* S, int64_t ld, hipStream_t s, const int* gate) {
  const Layout& L = v->L;
  lv_status st = LV_OK;
  for (int q = 1; q <= L.nsk && st == LV_OK; ++q) {
    double* prev = v->gT((L.m + q) & 1);
    double* next = v->gT((L.m + q + 1) & 1);
    st = hip_check(launch_gemm_rect<double>(S, ld, v->gB(), L.pp, v->gTmp(), L.pp, L.n_pad, L.pp, L.n_pad, s, gate),
                   "S_s B");
    if (st == LV_OK)
      st = hip_check(launch_gemm_rect<double>(P, ld, prev, L.pp, next, L.pp, L.n_pad, L.pp, L.n_pad, s, gate), "P_s T");
    if (st == LV_OK) st = hip_check(launch_add<double>(next, v->gTmp(), L.n_pad * L.pp, s, gate), "+ S_s B");
    if (st == LV_OK)
      st = hip_check(launch_copy_rect<double, T>(next, L.pp, L.n_pad, L.pp, v->Tskp<T>(q), L.n_pad, L.pp, s, gate),
                     "round T");
  }
  return st;
}

template <typename T>
lv_status build_chain(lv_view* v, hipStream_t s, const int* gate = nullptr) {
  const Layout& L = v->L;
  const int64_t cnt = L.n_pad * L.ldp;
  if (L.sums) {
    // S_1 = I (Sec. 5.2.3, Table 1)
    lv_status st = hip_check(launch_set_identity<T>(v->S<T>(0), L.ldp, v->n, L.n_pad, s, gate), "S_1 = I");
    if (st != LV_OK) return st;
  }
  if constexpr (sizeof(T) == 8) {
    if (L.general) {
      lv_status st = general_step<double>(v, 0, v->P<double>(0), nullptr, L.ldp, s, gate);
      if (st != LV_OK) return st;
    }
    for (int j = 1; j <= L.m; ++j) {
      if (L.general) {
        lv_status st = general_step<double>(v, j, v->P<double>(j - 1), v->S<double>(j - 1), L.ldp, s, gate);
        if (st != LV_OK) return st;
      }
      lv_status st = hip_check(launch_gemm<double>(v->P<double>(j - 1), L.ldp, v->P<double>(j - 1), L.ldp,
                                                   v->P<double>(j), L.ldp, L.n_pad, s, gate), "gemm f64");
      if (st != LV_OK) return st;
      if (L.sums) {
        // S_{2i} = P_i S_i + S_i
        st = hip_check(launch_gemm<double>(v->P<double>(j - 1), L.ldp, v->S<double>(j - 1), L.ldp, v->S<double>(j),
                                           L.ldp, L.n_pad, s, gate), "gemm f64 (sums)");
        if (st == LV_OK) st = hip_check(launch_add<double>(v->S<double>(j), v->S<double>(j - 1), cnt, s, gate), "S add");
        if (st != LV_OK) return st;
      }
    }
    if (L.nsk > 0) {
      lv_status st = skip_steps<double>(v, v->P<double>(L.m), v->S<double>(L.m), L.ldp, s, gate);
      if (st != LV_OK) return st;
    }
  } else {
    if (L.m == 0 && !L.general) return LV_OK;
    lv_status st = hip_check(launch_copy_pad<float, double>(v->P<float>(0), L.ldp, L.n_pad, v->scratch(0),
                                                            L.n_pad, L.n_pad, s, gate), "widen P_1");
    if (st == LV_OK && L.sums)
      st = hip_check(launch_set_identity<double>(v->sscratch(0), L.n_pad, v->n, L.n_pad, s, gate), "S_1 = I (f64)");
    if (st == LV_OK && L.general) st = general_step<float>(v, 0, v->scratch(0), nullptr, L.n_pad, s, gate);
    if (st != LV_OK) return st;
    for (int j = 1; j <= L.m; ++j) {
      double* src = v->scratch((j - 1) & 1);
      double* dst = v->scratch(j & 1);
      if (L.general) {
        st = general_step<float>(v, j, src, v->sscratch((j - 1) & 1), L.n_pad, s, gate);
        if (st != LV_OK) return st;
      }
      if (L.sums) {
        // S_{2i} = P_i S_i + S_i in double from the double P_i, rounded once
        double* scur = v->sscratch((j - 1) & 1);
        double* snew = v->sscratch(j & 1);
        st = hip_check(launch_gemm<double>(src, L.n_pad, scur, L.n_pad, snew, L.n_pad, L.n_pad, s, gate),
                       "gemm f64 (sums)");
        if (st == LV_OK) st = hip_check(launch_add<double>(snew, scur, (int64_t)L.n_pad * L.n_pad, s, gate), "S add");
        if (st == LV_OK)
          st = hip_check(launch_copy_pad<double, float>(snew, L.n_pad, L.n_pad, v->S<float>(j), L.ldp, L.n_pad, s,
                                                        gate),
                         "round S");
        if (st != LV_OK) return st;
      }
      st = hip_check(launch_gemm<double>(src, L.n_pad, src, L.n_pad, dst, L.n_pad, L.n_pad, s, gate),
                     "gemm f64");
      if (st != LV_OK) return st;
      st = hip_check(launch_copy_pad<double, float>(dst, L.n_pad, L.n_pad, v->P<float>(j), L.ldp, L.n_pad, s,
                                                    gate),
                     "round P");
      if (st != LV_OK) return st;
    }
    if (L.nsk > 0) {
      st = skip_steps<float>(v, v->scratch(L.m & 1), v->sscratch(L.m & 1), L.n_pad, s, gate);
      if (st != LV_OK) return st;
    }
    if (v->shadowed())
      for (int j = 0; j < L.m; ++j) {
        st = hip_check(launch_to_bf16(v->P<float>(j), v->shadow(j), L.n_pad * L.ldp, s, gate), "shadow");
        if (st != LV_OK) return st;
      }
  }
  return LV_OK;
}

// Drift check: P_j z for every level, P_j (P_j z) below the top, the
// residual kernel (gate + counter), then the gated squaring chain.
// `padded`: z already holds n_pad entries with zeros beyond n (the view's own
// probe vector of the periodic check); else it is the caller's n entries.
template <typename T>
lv_status drift_check(lv_view* v, const double* z, double tau, hipStream_t s, bool padded = false) {
  const Layout& L = v->L;
  lv_status st = padded ? LV_OK : hip_check(launch_vec_pad(z, v->n, v->zpad(), L.n_pad, s), "pad z");
  const double* zp = padded ? z : v->zpad();
  for (int j = 0; j <= L.m && st == LV_OK; ++j)
    st = hip_check(launch_matvec<T>(v->P<T>(j), L.ldp, L.n_pad, zp, v->Pz(j), s), "P z");
  for (int j = 0; j < L.m && st == LV_OK; ++j)
    st = hip_check(launch_matvec<T>(v->P<T>(j), L.ldp, L.n_pad, v->Pz(j), v->PPz(j), s), "P P z");
  if (st != LV_OK) return st;
  st = hip_check(launch_drift_residual(v->zpad() + L.n_pad, v->zpad() + (size_t)(L.m + 2) * L.n_pad, L.m,
                                       L.n_pad, tau, v->residuals(), v->gate(), v->drift_counter(), s),
                 "residual");
  if (st != LV_OK) return st;
  return build_chain<T>(v, s, v->gate());
}

}  // namespace

namespace lv {
lv_status periodic_drift(lv_view* v, hipStream_t s) {
  if (v->drift_every <= 0 || v->L.m == 0 || v->updates % v->drift_every != 0) return LV_OK;
  v->drift_checks += 1;
  return v->mode == LV_FP64 ? drift_check<double>(v, v->drift_z(), v->drift_tau, s, true)
                            : drift_check<float>(v, v->drift_z(), v->drift_tau, s, true);
}
}  // namespace lv

namespace {

hipEvent_t take_event(lv_view* v) {
  if (!v->pool.empty()) { hipEvent_t e = v->pool.back(); v->pool.pop_back(); return e; }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Runs `launch` and, when timing is on, brackets it with an event pair of
// the given kind (0 fused, 1 tail, 2 top update).
template <typename F>
lv_status timed(lv_view* v, int kind, hipStream_t s, const char* what, F&& launch) {
  hipEvent_t a = nullptr, b = nullptr;
  if (v->timing) {
    a = take_event(v);
    b = take_event(v);
    if (!a || !b) return fail(LV_EDEVICE, "hipEventCreate failed");
    if (hipEventRecord(a, s) != hipSuccess) return fail(LV_EDEVICE, "hipEventRecord failed");
  }
  lv_status st = hip_check(launch(), what);
  if (st != LV_OK) return st;
  if (v->timing) {
    if (hipEventRecord(b, s) != hipSuccess) return fail(LV_EDEVICE, "hipEventRecord failed");
    v->pending.push_back({a, b, kind});
  }
  return LV_OK;
}

// Sums of powers, level j after the powers' level step (the powers' partials
// of level j are consumed, so a pass may write its unused X there):
// Y_s = S_j^T V_j with the OLD S_j, G_s = Q_j^T V_j, S_j += Q_j W_j^T, and the
// sums tail (Q_{j+1}, W_{j+1}).  Below the matrix-core ranks Y_s and the
// update share one pass over S_j (launch_sums_fused); from float rank 16 up
// Y_s is a read-only pass on the matrix cores, then the update pass.  Level
// 0 has Q_0 = 0 and S_0 = I: only the tail runs.  (X_s = P_j Q_j came from
// the powers' pass or from its own read-only pass before it.)
template <typename T>
lv_status sums_level(lv_view* v, int j, int R, const T* sU, const T* sV, hipStream_t s) {
  const Layout& L = v->L;
  lv_status st = LV_OK;
  if (j > 0 && sums_fused(R, (int)sizeof(T))) {
    // one pass over S_j: Y = S_j^T V_j (old S_j), S_j += Q_j W_j^T
    st = timed(v, 0, s, "sums: pass", [&] {
      return launch_sums_fused<T>(R, v->S<T>(j), L.ldp, L.n_pad, v->tile_rows[j], v->slabQ<T>(), v->slabW<T>(), sV,
                                  L.W, v->partYs<T>(j), s);
    });
    if (st == LV_OK)
      st = timed(v, 0, s, "sums: gram", [&] {
        return launch_gram_cols<T>(R, sV + (L.W - R), v->slabQ<T>(), L.W, L.n_pad, v->partGs(j), s);
      });
    if (st != LV_OK) return st;
  } else if (j > 0) {
    st = timed(v, 0, s, "sums: S^T V", [&] {
      if (skinny_on_mfma(R, (int)sizeof(T)))
        return launch_skinny_f32(R, reinterpret_cast<const float*>(v->S<T>(j)), L.ldp, L.n_pad, v->tile_rows[j],
                                 v->slabQ<float>(), reinterpret_cast<const float*>(sV), L.W,
                                 reinterpret_cast<float*>(v->partX<T>(j)), v->partYs<float>(j), s, kWantY);
      return launch_level_readonly<T>(R, v->S<T>(j), L.ldp, L.n_pad, v->tile_rows[j], v->slabQ<T>(),
                                      sV + (L.W - R), L.W, v->partX<T>(j), v->partYs<T>(j), s);
    });
    if (st == LV_OK)
      st = timed(v, 0, s, "sums: gram", [&] {
        return launch_gram_cols<T>(R, sV + (L.W - R), v->slabQ<T>(), L.W, L.n_pad, v->partGs(j), s);
      });
    if (st == LV_OK)
      st = timed(v, 0, s, "sums: update", [&] {
        return launch_level_update<T>(R, v->S<T>(j), L.ldp, L.n_pad, v->slabQ<T>(), v->slabW<T>(), L.W, s);
      });
    if (st != LV_OK) return st;
  }
  return timed(v, 1, s, "sums: tail", [&] {
    return launch_sums_tail<T>(R, v->partXs<T>(j), v->partYs<T>(j), v->partGs(j), L.nct, v->nrt(j), L.n_pad,
                               v->slabQ<T>(), v->slabW<T>(), sU, sV, L.W, j == 0, s);
  });
}

// General form, level j (hybrid deltas, D_{2^j} in D[j & 1]): the product
// X = P_j D_j with the OLD P_j, run before the level's update.  Float from
// rank 16 up on the matrix cores (X only), else the read-only vector pass
// (its transposed product is discarded).
template <typename T>
lv_status general_pass(lv_view* v, int j, hipStream_t s) {
  const Layout& L = v->L;
  const T* Dj = v->D<T>(j & 1);
  return timed(v, 0, s, "general: P D", [&] {
    if (skinny_on_mfma(L.pp, (int)sizeof(T)))
      return launch_skinny_f32(L.pp, reinterpret_cast<const float*>(v->P<T>(j)), L.ldp, L.n_pad, v->tile_rows[j],
                               reinterpret_cast<const float*>(Dj), reinterpret_cast<const float*>(Dj), L.pp,
                               v->partXT<float>(), v->partYT<float>(), s, kWantX);
    return launch_level_readonly<T>(L.pp, v->P<T>(j), L.ldp, L.n_pad, v->tile_rows[j], Dj, Dj, L.pp,
                                    v->partXT<T>(), v->partYT<T>(), s);
  });
}

// General form, rest of level j, after the powers' tail (U_j, V_j intact)
// and before the sums tail (which overwrites Q_j):
// a = V_j^T T_{2^j} (T_{2^j} already holds T + D), b = W_j^T B (j > 0,
// W_0 = 0), D_{2^(j+1)} = X + U_j a + Q_j b, T_{2^(j+1)} += D.  With
// j < 0 the first step: D_1 = U (V^T T_0), T_1 += D_1.
template <typename T>
lv_status general_tail(lv_view* v, int j, int R, const T* sU, const T* sV, hipStream_t s) {
  const Layout& L = v->L;
  const bool first = j < 0;
  const T* src = first ? v->T0<T>() : v->Tg<T>(j);
  lv_status st = timed(v, 0, s, "general: V^T T", [&] {
    return launch_atb<T>(R, L.pp, sV + (L.W - R), L.W, src, L.pp, L.n_pad, v->atbA(), s);
  });
  if (st == LV_OK && j > 0)
    st = timed(v, 0, s, "general: W^T B", [&] {
      return launch_atb<T>(R, L.pp, v->slabW<T>() + (L.W - R), L.W, v->Bg<T>(), L.pp, L.n_pad, v->atbB(), s);
    });
  if (st != LV_OK) return st;
  return timed(v, 1, s, "general: tail", [&] {
    return launch_general_tail<T>(v->partXT<T>(), first ? 0 : L.nct, sU, j > 0 ? v->slabQ<T>() : nullptr, L.W, R,
                                  v->atbA(), v->atbB(), v->D<T>((j + 1) & 1), v->Tg<T>(j + 1), L.n_pad, L.pp, s);
  });
}

// Widths of the factored deltas for an update of padded rank ru (the slabs
// are laid out for r_max; their columns beyond these widths are zero):
// Y_j, Z_j have (2^(j+1) - 1) ru columns, the skip factors wy(m) + 2 q ru 2^m.
inline int gw(int ru, int j) { return ((2 << j) - 1) * ru; }
inline int gW(int ru, int j) { return (int)next_pow2(gw(ru, j)); }
inline int gwsk(const Layout& L, int ru, int q) { return gw(ru, L.m) + q * 2 * (ru << L.m); }
inline int gWsk(const Layout& L, int ru, int q) { return (int)next_pow2(gwsk(L, ru, q)); }

// General form with factored deltas Delta T_j = Y_j Z_j^T (App. B,
// exponential model): Y_0 is the prefix [0, r_pad) of the powers' U slab,
// Z_0 = T_0^T V.  Every T_j keeps its old value until the whole update has
// formed its factors (gfac_finish applies T_j += Y_j Z_j^T).
template <typename T>
lv_status gfac_first(lv_view* v, int ru, const T* sV, hipStream_t s) {
  const Layout& L = v->L;
  lv_status st = timed(v, 0, s, "general: T_0^T V", [&] {
    return launch_atb<T>(ru, L.pp, sV + (L.W - ru), L.W, v->T0<T>(), L.pp, L.n_pad, v->atbA(), s);
  });
  if (st != LV_OK) return st;
  return timed(v, 1, s, "general: Z_0", [&] {
    return launch_gfac_z<T>(v->atbA(), nullptr, 0, nullptr, ru, v->Ztf<T>(0), L.WY[0], L.pp, s);
  });
}

// Level j, before the powers' update: X = P_j Y_j with the OLD P_j (the
// float matrix cores from width 16, X only; else the read-only vector pass).
template <typename T>
lv_status gfac_pass(lv_view* v, int j, int ru, const T* sU, hipStream_t s) {
  const Layout& L = v->L;
  const T* Yj = j == 0 ? sU : v->Yf<T>(j);
  const int sy = j == 0 ? L.W : L.WY[j];
  const int R = gW(ru, j);
  return timed(v, 0, s, "general: P Y", [&] {
    if (skinny_on_mfma(R, (int)sizeof(T)))
      return launch_skinny_f32(R, reinterpret_cast<const float*>(v->P<T>(j)), L.ldp, L.n_pad, v->tile_rows[j],
                               reinterpret_cast<const float*>(Yj), reinterpret_cast<const float*>(Yj), sy,
                               v->partXT<float>(), v->partYT<float>(), s, kWantX);
    return launch_level_readonly<T>(R, v->P<T>(j), L.ldp, L.n_pad, v->tile_rows[j], Yj, Yj, sy, v->partXT<T>(),
                                    v->partYT<T>(), s);
  });
}

// Level j, after the powers' tail (U_j, V_j intact) and before the sums'
// tail (Q_j intact): G = V_j^T Y_j, a = V_j^T T_j (old T_j), b = W_j^T B
// (j > 0), then Y_{j+1} = [U_j, X + U_j G, Q_j] and Z_{j+1}^T = [a; Z_j^T; b].
template <typename T>
lv_status gfac_tail(lv_view* v, int j, int R, int ru, const T* sU, const T* sV, hipStream_t s) {
  const Layout& L = v->L;
  const T* Yj = j == 0 ? sU : v->Yf<T>(j);
  const int sy = j == 0 ? L.W : L.WY[j];
  const int wj = gW(ru, j);
  const T* Vj = sV + (L.W - R);
  lv_status st = timed(v, 0, s, "general: V^T Y", [&] {
    return launch_atb<T>(R, wj, Vj, L.W, Yj, sy, L.n_pad, v->atbG(), s);
  });
  if (st == LV_OK)
    st = timed(v, 0, s, "general: V^T T", [&] {
      return launch_atb<T>(R, L.pp, Vj, L.W, v->Tg<T>(j), L.pp, L.n_pad, v->atbA(), s);
    });
  if (st == LV_OK && j > 0)
    st = timed(v, 0, s, "general: W^T B", [&] {
      return launch_atb<T>(R, L.pp, v->slabW<T>() + (L.W - R), L.W, v->Bg<T>(), L.pp, L.n_pad, v->atbB(), s);
    });
  if (st == LV_OK)
    st = timed(v, 1, s, "general: Y", [&] {
      // X = P_j Y_j: at level 0 (Y_0 = U_0) the partials of the powers' pass
      return launch_gfac_y<T>(j == 0 ? v->partX<T>(0) : v->partXT<T>(), L.nct, wj, sU, j > 0 ? v->slabQ<T>() : nullptr,
                              L.W, R, v->atbG(), wj, gw(ru, j), v->Yf<T>(j + 1), L.WY[j + 1], L.n_pad, s);
    });
  if (st == LV_OK)
    st = timed(v, 1, s, "general: Z", [&] {
      return launch_gfac_z<T>(v->atbA(), v->Ztf<T>(j), gw(ru, j), j > 0 ? v->atbB() : nullptr, R, v->Ztf<T>(j + 1),
                              L.WY[j + 1], L.pp, s);
    });
  return st;
}

// Skip model (Table 1; App. B skip model, factored): for q = 1 .. nsk,
// T_{(q+1)s} = P_s T_{qs} + S_s B gives, with the OLD P_s, T_{qs} and the
// top-level factors U_s, V_s, Q_s, W_s (all formed by the level loop),
//   Y = [U_s, P_s Y_prev + U_s (V_s^T Y_prev), Q_s],  Z = [T_prev^T V_s, Z_prev, B^T W_s].
// Runs before the top update of P_s.
template <typename T>
lv_status gfac_skip(lv_view* v, int ru, const T* sU, const T* sV, hipStream_t s) {
  const Layout& L = v->L;
  const int Rm = ru << L.m;
  const T* Vm = sV + (L.W - Rm);
  lv_status st = LV_OK;
  if (L.m > 0)
    st = timed(v, 0, s, "general: W_s^T B", [&] {
      return launch_atb<T>(Rm, L.pp, v->slabW<T>() + (L.W - Rm), L.W, v->Bg<T>(), L.pp, L.n_pad, v->atbB(), s);
    });
  for (int q = 1; q <= L.nsk && st == LV_OK; ++q) {
    const T* Yp = q > 1 ? v->Yskp<T>(q - 1) : (L.m == 0 ? sU : v->Yf<T>(L.m));
    const int sp = q > 1 ? L.WYsk(q - 1) : (L.m == 0 ? L.W : L.WY[L.m]);
    const int wp = q > 1 ? gWsk(L, ru, q - 1) : gW(ru, L.m);
    const T* Zp = q > 1 ? v->Ztskp<T>(q - 1) : v->Ztf<T>(L.m);
    const T* Tp = q > 1 ? v->Tskp<T>(q - 1) : v->Tg<T>(L.m);
    st = timed(v, 0, s, "general: P_s Y", [&] {
      if (skinny_on_mfma(wp, (int)sizeof(T)))
        return launch_skinny_f32(wp, reinterpret_cast<const float*>(v->P<T>(L.m)), L.ldp, L.n_pad, kTileRows,
                                 reinterpret_cast<const float*>(Yp), reinterpret_cast<const float*>(Yp), sp,
                                 v->partXT<float>(), v->partYT<float>(), s, kWantX);
      return launch_level_readonly<T>(wp, v->P<T>(L.m), L.ldp, L.n_pad, kTileRows, Yp, Yp, sp, v->partXT<T>(),
                                      v->partYT<T>(), s);
    });
    if (st == LV_OK)
      st = timed(v, 0, s, "general: V_s^T Y", [&] {
        return launch_atb<T>(Rm, wp, Vm, L.W, Yp, sp, L.n_pad, v->atbG(), s);
      });
    if (st == LV_OK)
      st = timed(v, 0, s, "general: V_s^T T", [&] {
        return launch_atb<T>(Rm, L.pp, Vm, L.W, Tp, L.pp, L.n_pad, v->atbA(), s);
      });
    if (st == LV_OK)
      st = timed(v, 1, s, "general: Y (skip)", [&] {
        return launch_gfac_y<T>(v->partXT<T>(), L.nct, wp, sU, L.m > 0 ? v->slabQ<T>() : nullptr, L.W, Rm,
                                v->atbG(), wp, gwsk(L, ru, q - 1), v->Yskp<T>(q), L.WYsk(q), L.n_pad, s);
      });
    if (st == LV_OK)
      st = timed(v, 1, s, "general: Z (skip)", [&] {
        return launch_gfac_z<T>(v->atbA(), Zp, gwsk(L, ru, q - 1), L.m > 0 ? v->atbB() : nullptr, Rm, v->Ztskp<T>(q),
                                L.WYsk(q), L.pp, s);
      });
  }
  return st;
}

template <typename T>
lv_status gfac_finish(lv_view* v, int ru, const T* sU, hipStream_t s) {
  const Layout& L = v->L;
  lv_status st = LV_OK;
  for (int j = 0; j <= L.m && st == LV_OK; ++j)
    st = timed(v, 2, s, "general: T += Y Z^T", [&] {
      return launch_rank_rect<T>(v->Tg<T>(j), j == 0 ? sU : v->Yf<T>(j), j == 0 ? L.W : L.WY[j], v->Ztf<T>(j),
                                 gw(ru, j), L.n_pad, L.pp, s);
    });
  for (int q = 1; q <= L.nsk && st == LV_OK; ++q)
    st = timed(v, 2, s, "general: T += Y Z^T (skip)", [&] {
      return launch_rank_rect<T>(v->Tskp<T>(q), v->Yskp<T>(q), L.WYsk(q), v->Ztskp<T>(q), gwsk(L, ru, q), L.n_pad,
                                 L.pp, s);
    });
  return st;
}

// Level j of one update (App. A exponential model; trigger of Sec. 4.4) with
// the update's factors in the slabs sU, sV: the fused pass and the tail (or,
// for float storage at large level rank and with bfloat16 shadows, the
// read-only skinny pass, the Gram and the update pass), then the sums' and
// the general form's level steps.  Stream-ordered on s.
template <typename T>
lv_status level_step(lv_view* v, int j, int r_pad, T* sU, T* sV, hipStream_t s, bool pipelined = false) {
  const Layout& L = v->L;
  lv_status st = LV_OK;
  const int R = r_pad << j;
  // The general form's product with the OLD P_j: P_j D_j (hybrid) or P_j Y_j
  // (factored; at level 0 Y_0 = U_0, so the powers' own X serves).  It
  // rides on the powers' fused pass when the X width allows, like P_j Q_j
  // of the sums; else it is a read-only pass of its own.
  const bool gen_op = L.general && !(L.gfac && j == 0);
  const bool vec_level = fused_vector_level(R, (int)sizeof(T), v->shadowed());
  const bool q_in_pass = L.sums && j > 0 && vec_level && fused_extra_fits(R, true, 0);
  const int xd = !gen_op ? 0 : L.gfac ? gW(r_pad, j) : L.pp;
  const bool d_in_pass = gen_op && vec_level && fused_extra_fits(R, q_in_pass, xd);
  if (gen_op && !d_in_pass) {
    st = L.gfac ? gfac_pass<T>(v, j, r_pad, sU, s) : general_pass<T>(v, j, s);
    if (st != LV_OK) return st;
  }
  if (L.sums && j > 0 && !q_in_pass) {
    // sums: X_s = P_j Q_j with the OLD P_j, before this level's update
    st = timed(v, 0, s, "sums: P Q", [&] {
      if (skinny_on_mfma(R, (int)sizeof(T)))
        return launch_skinny_f32(R, reinterpret_cast<const float*>(v->P<T>(j)), L.ldp, L.n_pad, v->tile_rows[j],
                                 v->slabQ<float>(), reinterpret_cast<const float*>(sV), L.W, v->partXs<float>(j),
                                 v->partYs<float>(j), s, kWantX);
      return launch_level_readonly<T>(R, v->P<T>(j), L.ldp, L.n_pad, v->tile_rows[j], v->slabQ<T>(),
                                      sV + (L.W - R), L.W, v->partXs<T>(j), v->partYs<T>(j), s);
    });
    if (st != LV_OK) return st;
  }
  bool on_cores = false;
  if constexpr (sizeof(T) == 4) {
    if (v->shadowed() || skinny_on_mfma(R, 4)) {
      on_cores = true;
      // read-only skinny pass on the matrix cores (from the shadow, or from
      // the float power), FP64 Gram, then the rank update (which rewrites
      // the shadow after the skinny pass has read it); with the float power
      // at R = 16 the skinny pass applies the update itself (one read of
      // P_j), else the update pass follows
      const bool fused_upd = !v->shadowed() && skinny_fuses_update(R);
      st = timed(v, 0, s, "skinny", [&] {
        return v->shadowed() ? launch_skinny_bf16(R, v->shadow(j), L.ldp, L.n_pad, v->tile_rows[j], sU, sV, L.W,
                                                  v->partX<float>(j), v->partY<float>(j), s)
                             : launch_skinny_f32(R, v->P<float>(j), L.ldp, L.n_pad, v->tile_rows[j], sU, sV, L.W,
                                                 v->partX<float>(j), v->partY<float>(j), s, kWantX | kWantY,
                                                 fused_upd);
      });
      if (st == LV_OK)
        st = timed(v, 0, s, "gram", [&] {
          return launch_level_gram<float>(R, sU, sV, L.W, L.n_pad, v->partG(j), s);
        });
      if (st == LV_OK && !fused_upd)
        st = timed(v, 0, s, "update", [&] {
          return launch_level_update<float>(R, v->P<float>(j), L.ldp, L.n_pad, sU, sV, L.W, s,
                                            v->shadowed() ? v->shadow(j) : nullptr, v->shadowed());
        });
      if (st == LV_OK)
        st = timed(v, 1, s, "level tail", [&] {
          return launch_level_tail<float>(R, v->partX<float>(j), v->partY<float>(j), v->partG(j), L.nct, v->nrt(j),
                                          1, L.n_pad, sU, sV, L.W, s);
        });
    }
  }
  if (!on_cores) {
    st = timed(v, 0, s, "level pass", [&] {
      if (q_in_pass || d_in_pass) {
        const T* Dop = !d_in_pass ? nullptr : L.gfac ? v->Yf<T>(j) : v->D<T>(j & 1);
        const int ldd = L.gfac ? L.WY[j] : L.pp;
        return launch_level_fused_x<T>(R, v->P<T>(j), L.ldp, L.n_pad, v->tile_rows[j], sU, sV, L.W, v->partX<T>(j),
                                       v->partY<T>(j), v->partG(j), q_in_pass ? v->slabQ<T>() : nullptr,
                                       v->partXs<T>(j), Dop, ldd, d_in_pass ? xd : 0, v->partXT<T>(), s);
      }
      return launch_level_fused<T>(R, v->P<T>(j), L.ldp, L.n_pad, v->tile_rows[j], sU, sV, L.W, v->partX<T>(j),
                                   v->partY<T>(j), v->partG(j), s,
                                   pipelined ? pipe_slice_groups(L.nct, v->nrt(j)) : 0);
    });
    if (st == LV_OK)
      st = timed(v, 1, s, "level tail", [&] {
        return launch_level_tail<T>(R, v->partX<T>(j), v->partY<T>(j), v->partG(j), L.nct, v->nrt(j),
                                    gram_in_pass(R, (int)sizeof(T)) ? v->nrt(j) : 1, L.n_pad, sU, sV, L.W, s);
      });
  }
  if (st == LV_OK && L.general)
    st = L.gfac ? gfac_tail<T>(v, j, R, r_pad, sU, sV, s) : general_tail<T>(v, j, R, sU, sV, s);
  if (st == LV_OK && L.sums) st = sums_level<T>(v, j, R, sU, sV, s);
  return st;
}

// The update-only pass of the top stored power P_m with U_m, V_m.
template <typename T>
lv_status top_step(lv_view* v, int r_pad, T* sU, T* sV, hipStream_t s) {
  const Layout& L = v->L;
  const int Rm = r_pad << L.m;
  return timed(v, 2, s, "top update", [&] {
    return launch_level_update<T>(Rm, v->P<T>(L.m), L.ldp, L.n_pad, sU, sV, L.W, s, nullptr, v->shadowed());
  });
}

// One update through every level, factors in the view's slabs (App. A
// exponential model; trigger of Sec. 4.4): the level steps 0..m-1, then the
// top level's update-only pass.
template <typename T>
lv_status update_one(lv_view* v, const T* U, const T* V, int r, int64_t ldu, int64_t ldv,
                     hipStream_t s) {
  const Layout& L = v->L;
  const int r_pad = (int)next_pow2(r);
  T* sU = v->slabU<T>();
  T* sV = v->slabV<T>();
  lv_status st = hip_check(launch_prep<T>(U, ldu, V, ldv, v->n, r, r_pad, sU, sV, L.W, L.n_pad, s), "prep");
  if (st == LV_OK && L.general)
    st = L.gfac ? gfac_first<T>(v, r_pad, sV, s) : general_tail<T>(v, -1, r_pad, sU, sV, s);
  for (int j = 0; j < L.m && st == LV_OK; ++j) st = level_step<T>(v, j, r_pad, sU, sV, s);
  if (st == LV_OK && L.nsk > 0) st = gfac_skip<T>(v, r_pad, sU, sV, s);
  if (st == LV_OK) st = top_step<T>(v, r_pad, sU, sV, s);
  if (st == LV_OK && L.sums && L.m > 0)
    st = timed(v, 2, s, "sums: top update", [&] {
      return launch_level_update<T>(r_pad << L.m, v->S<T>(L.m), L.ldp, L.n_pad, v->slabQ<T>(), v->slabW<T>(), L.W,
                                    s);
    });
  if (st == LV_OK && L.gfac) st = gfac_finish<T>(v, r_pad, sU, s);
  return st;
}

// Pipelined batch of updates (plain views: no sums, no general form).  Level
// j of update t needs only P_j as update t-1 left it and the factors that
// level j-1 of update t assembled, so the levels are cut into stages
// (contiguous level ranges, at most kPipeStreams), each on a stream of its
// own (stage 0 on the caller's stream), and successive updates flow through
// them: while a stage works on update t the earlier stages already work on
// t+1, t+2, ...  Each update in flight holds one of pipe_slots factor-slab
// pairs; a slab is reused only after the top level of the update that held
// it has finished.  Every kernel sees exactly the inputs of the sequential
// order, so the results are bit-identical to it.
inline int pipe_stage(const lv_view* v, int j) { return j * v->pipe_nstages / v->L.m; }

lv_status pipe_setup(lv_view* v) {
  if (v->pipe_nstages > 0) return LV_OK;
  const int ns = v->L.m < kPipeStreams ? v->L.m : kPipeStreams;
  for (int q = 1; q < ns; ++q)
    if (hipStreamCreateWithFlags(&v->pstream[q], hipStreamNonBlocking) != hipSuccess)
      return fail(LV_EDEVICE, "hipStreamCreateWithFlags failed");
  auto mk = [](hipEvent_t* e) { return hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess; };
  bool ok = mk(&v->pfork);
  for (int q = 0; q < ns && ok; ++q) ok = mk(&v->pjoin[q]);
  for (int sl = 0; sl < v->L.pipe_slots && ok; ++sl) {
    ok = mk(&v->pfree[sl]);
    for (int j = 0; j + 1 < v->L.m && ok; ++j) ok = mk(&v->pready[j][sl]);
  }
  if (!ok) return fail(LV_EDEVICE, "hipEventCreateWithFlags failed");
  v->pipe_nstages = ns;
  return LV_OK;
}

// The stage streams wait for the caller's stream (fork) or the caller's
// stream for every stage (join).
lv_status pipe_fork(lv_view* v, hipStream_t s) {
  if (hipEventRecord(v->pfork, s) != hipSuccess) return fail(LV_EDEVICE, "hipEventRecord failed");
  for (int q = 1; q < v->pipe_nstages; ++q)
    if (hipStreamWaitEvent(v->pstream[q], v->pfork, 0) != hipSuccess) return fail(LV_EDEVICE, "hipStreamWaitEvent failed");
  return LV_OK;
}

lv_status pipe_join(lv_view* v, hipStream_t s) {
  for (int q = 1; q < v->pipe_nstages; ++q) {
    if (hipEventRecord(v->pjoin[q], v->pstream[q]) != hipSuccess) return fail(LV_EDEVICE, "hipEventRecord failed");
    if (hipStreamWaitEvent(s, v->pjoin[q], 0) != hipSuccess) return fail(LV_EDEVICE, "hipStreamWaitEvent failed");
  }
  return LV_OK;
}

template <typename T>
lv_status update_batch_pipelined(lv_view* v, const char* U, const char* V, int r, int64_t count, int64_t ldu,
                                 int64_t ldv, int64_t strideU, int64_t strideV, hipStream_t s) {
  const Layout& L = v->L;
  lv_status st = pipe_setup(v);
  if (st != LV_OK) return st;
  st = pipe_fork(v, s);
  if (st != LV_OK) return st;
  const int r_pad = (int)next_pow2(r);
  const int D = L.pipe_slots;
  auto stream_of = [&](int j) { const int q = pipe_stage(v, j); return q == 0 ? s : v->pstream[q]; };
  auto ev = [&](hipError_t e, const char* what) { return e == hipSuccess ? LV_OK : fail(LV_EDEVICE, "%s failed", what); };
  for (int64_t t = 0; t < count && st == LV_OK; ++t) {
    const int sl = (int)(t % D);
    T* sU = v->slabU<T>(sl);
    T* sV = v->slabV<T>(sl);
    const T* Ut = reinterpret_cast<const T*>(U + (size_t)(t * strideU) * sizeof(T));
    const T* Vt = reinterpret_cast<const T*>(V + (size_t)(t * strideV) * sizeof(T));
    // the slab is free once the top level of update t - D is done with it
    if (t >= D) st = ev(hipStreamWaitEvent(s, v->pfree[sl], 0), "hipStreamWaitEvent");
    if (st == LV_OK) st = hip_check(launch_prep<T>(Ut, ldu, Vt, ldv, v->n, r, r_pad, sU, sV, L.W, L.n_pad, s), "prep");
    for (int j = 0; j < L.m && st == LV_OK; ++j) {
      hipStream_t sj = stream_of(j);
      if (j > 0 && pipe_stage(v, j - 1) != pipe_stage(v, j))
        st = ev(hipStreamWaitEvent(sj, v->pready[j - 1][sl], 0), "hipStreamWaitEvent");
      if (st == LV_OK) st = level_step<T>(v, j, r_pad, sU, sV, sj, true);
      if (st == LV_OK && j + 1 < L.m && pipe_stage(v, j + 1) != pipe_stage(v, j))
        st = ev(hipEventRecord(v->pready[j][sl], sj), "hipEventRecord");
    }
    hipStream_t st_top = stream_of(L.m - 1);
    if (st == LV_OK) st = top_step<T>(v, r_pad, sU, sV, st_top);
    if (st == LV_OK) st = ev(hipEventRecord(v->pfree[sl], st_top), "hipEventRecord");
    if (st != LV_OK) break;
    v->updates += 1;
    if (v->drift_every > 0 && v->updates % v->drift_every == 0) {
      // the drift check reads every power: all stages join, then fork again
      st = pipe_join(v, s);
      if (st == LV_OK) st = periodic_drift(v, s);
      if (st == LV_OK) st = pipe_fork(v, s);
    }
  }
  const lv_status sj = pipe_join(v, s);
  return st != LV_OK ? st : sj;
}

// ---------------------------------------------------------------- re-evaluation
//
// Workspace: two n_pad x n_pad ping-pong matrices and one factor slab pair
// (n_pad x r_pad each).

size_t reeval_bytes(int64_t n_pad, int r_pad, int elem) {
  return 2 * align_up((size_t)n_pad * n_pad * elem) + 2 * align_up((size_t)n_pad * r_pad * elem);
}

template <typename T>
lv_status reeval_impl(const T* A, int64_t n, int64_t lda, int k, const T* U, const T* V, int r,
                             int64_t ldu, int64_t ldv, T* out, int64_t ldo, char* ws, hipStream_t s) {
  const int64_t n_pad = round_up(n, kPadOrder);
  const int r_pad = (int)next_pow2(r < 1 ? 1 : r);
  const size_t mat = align_up((size_t)n_pad * n_pad * sizeof(T));
  T* buf[2] = {reinterpret_cast<T*>(ws), reinterpret_cast<T*>(ws + mat)};
  T* sU = reinterpret_cast<T*>(ws + 2 * mat);
  T* sV = reinterpret_cast<T*>(ws + 2 * mat + align_up((size_t)n_pad * r_pad * sizeof(T)));
  lv_status st = hip_check(launch_copy_pad<T, T>(A, lda, n, buf[0], n_pad, n_pad, s), "copy A");
  if (st != LV_OK) return st;
  if (r > 0) {
    st = hip_check(launch_prep<T>(U, ldu, V, ldv, n, r, r_pad, sU, sV, r_pad, n_pad, s), "prep");
    if (st != LV_OK) return st;
    st = hip_check(launch_level_update<T>(r_pad, buf[0], n_pad, n_pad, sU, sV, r_pad, s), "A += U V^T");
    if (st != LV_OK) return st;
  }
  int cur = 0;
  for (int j = 1; (1 << j) <= k; ++j) {
    st = hip_check(launch_gemm<T>(buf[cur], n_pad, buf[cur], n_pad, buf[cur ^ 1], n_pad, n_pad, s), "gemm");
    if (st != LV_OK) return st;
    cur ^= 1;
  }
  return hip_check(hipMemcpy2DAsync(out, ldo * sizeof(T), buf[cur], n_pad * sizeof(T), n * sizeof(T), n,
                                    hipMemcpyDeviceToDevice, s), "copy out");
}

}  // namespace

extern "C" {

const char* lv_status_str(lv_status s) {
  switch (s) {
    case LV_OK: return "LV_OK";
    case LV_EINVAL: return "LV_EINVAL";
    case LV_ENOMEM: return "LV_ENOMEM";
    case LV_EDEVICE: return "LV_EDEVICE";
    case LV_ESTATE: return "LV_ESTATE";
  }
  return "LV_UNKNOWN";
}

const char* lv_last_error(void) { return g_err; }

size_t lv_view_footprint_ex(int64_t n, int k, int r_max, lv_mode mode, int flags) {
  if (check_shape(n, k, r_max, mode, flags == 0) != LV_OK || (flags & ~LV_WITH_SUMS) != 0) return 0;
  return make_layout(n, k, r_max, mode, flags).total;
}

size_t lv_view_footprint(int64_t n, int k, int r_max, lv_mode mode) {
  return lv_view_footprint_ex(n, k, r_max, mode, 0);
}

lv_status lv_view_create(const void* A, int64_t n, int64_t lda, int k, int r_max, lv_mode mode,
                         void* workspace, size_t ws_bytes, void* stream, lv_view** out) {
  return lv_view_create_ex(A, n, lda, k, r_max, mode, 0, workspace, ws_bytes, stream, out);
}

}  // extern "C"

namespace {

// Creation of every kind of view; p > 0 makes a general-form view with T_0
// and B (n x p, leading dimensions ldt, ldb).
lv_status create_view(const void* A, int64_t n, int64_t lda, int k, int r_max, lv_mode mode, int flags, int p,
                      bool factored, int kT, const void* T0, int64_t ldt, const void* B, int64_t ldb, void* workspace,
                      size_t ws_bytes, void* stream, lv_view** out) {
  g_err[0] = 0;
  if (!out) return fail(LV_EINVAL, "out is NULL");
  *out = nullptr;
  lv_status st = check_shape(n, k, r_max, mode, flags == 0 && p == 0);
  if (st != LV_OK) return st;
  if ((flags & ~LV_WITH_SUMS) != 0) return fail(LV_EINVAL, "unknown creation flags 0x%x", flags);
  if (!A || !workspace) return fail(LV_EINVAL, "A or workspace is NULL");
  if (lda < n) return fail(LV_EINVAL, "lda = %lld < n = %lld", (long long)lda, (long long)n);
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
    return fail(LV_ENOMEM, "workspace is not %zu-byte aligned", kAlign);
  const Layout L = make_layout(n, k, r_max, mode, flags, p, factored, kT);
  if (ws_bytes < L.total)
    return fail(LV_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
  lv_view* v = new (std::nothrow) lv_view();
  if (!v) return fail(LV_ENOMEM, "host allocation of the view handle failed");
  v->n = n; v->k = k; v->r_max = r_max; v->mode = mode; v->L = L;
  v->base = static_cast<char*>(workspace); v->ws_bytes = ws_bytes;
  v->updates = 0; v->reanchors = 0;
  for (int j = 0; j < kMaxLevel; ++j) v->tile_rows[j] = L.tile_rows;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (L.sums) {
    // the sum factor slabs start at zero: the W columns of level 0 are read as
    // W_0 = 0 and are never written afterwards
    st = hip_check(hipMemsetAsync(v->base + L.slabQ, 0, L.slabW - L.slabQ, s), "clear Q slab");
    if (st == LV_OK)
      st = hip_check(hipMemsetAsync(v->base + L.slabW, 0, (size_t)L.n_pad * L.W * L.elem, s), "clear W slab");
    if (st != LV_OK) { delete v; return st; }
  }
  if (mode == LV_FP64) {
    st = hip_check(launch_copy_pad<double, double>(static_cast<const double*>(A), lda, n, v->P<double>(0),
                                                   L.ldp, L.n_pad, s), "copy A");
    if (st == LV_OK && L.general)
      st = hip_check(launch_copy_rect<double, double>(static_cast<const double*>(T0), ldt, n, p, v->T0<double>(),
                                                      L.n_pad, L.pp, s), "copy T_0");
    if (st == LV_OK && L.general)
      st = hip_check(launch_copy_rect<double, double>(static_cast<const double*>(B), ldb, n, p, v->Bg<double>(),
                                                      L.n_pad, L.pp, s), "copy B");
    if (st == LV_OK) st = build_chain<double>(v, s);
  } else {
    st = hip_check(launch_copy_pad<float, float>(static_cast<const float*>(A), lda, n, v->P<float>(0),
                                                 L.ldp, L.n_pad, s), "copy A");
    if (st == LV_OK && L.general)
      st = hip_check(launch_copy_rect<float, float>(static_cast<const float*>(T0), ldt, n, p, v->T0<float>(),
                                                    L.n_pad, L.pp, s), "copy T_0");
    if (st == LV_OK && L.general)
      st = hip_check(launch_copy_rect<float, float>(static_cast<const float*>(B), ldb, n, p, v->Bg<float>(),
                                                    L.n_pad, L.pp, s), "copy B");
    if (st == LV_OK) st = build_chain<float>(v, s);
  }
  if (st == LV_OK)
    st = hip_check(hipMemsetAsync(v->gate(), 0, 128, s), "clear drift counters");
  if (st == LV_OK)
    st = hip_check(hipMemsetAsync(v->base + L.zfac, 0, (size_t)L.n_pad * L.r_pad * L.elem, s), "clear zero factors");
  if (st != LV_OK) { delete v; return st; }
  *out = v;
  return LV_OK;
}

}  // namespace

extern "C" {

lv_status lv_view_create_ex(const void* A, int64_t n, int64_t lda, int k, int r_max, lv_mode mode, int flags,
                            void* workspace, size_t ws_bytes, void* stream, lv_view** out) {
  return create_view(A, n, lda, k, r_max, mode, flags, 0, false, 0, nullptr, 0, nullptr, 0, workspace, ws_bytes,
                     stream, out);
}

}  // extern "C"

namespace {

// k iterations of T; the powers and sums run to s (s = 0 or s = k: the
// exponential model; else the skip-s model, factored deltas only).
lv_status check_general(int64_t n, int k, int r_max, lv_mode mode, int64_t p, int strategy, int s) {
  if (s != 0 && s != k) {
    if (strategy != LV_GENERAL_FACTORED) return fail(LV_EINVAL, "the skip model needs factored deltas");
    if (!is_pow2(s) || s > k || k % s != 0 || k > kMaxK)
      return fail(LV_EINVAL, "the skip model needs s a power of two dividing k, got s = %d, k = %d", s, k);
    const int64_t r_pad = next_pow2(r_max);
    // the widest operand of a P_s pass: (2k - 1 - 2s) r_pad columns
    if ((int64_t)(2 * k - 1 - 2 * s) * r_pad > 128 || (int64_t)(2 * k - 1) * r_pad > 256)
      return fail(LV_EINVAL, "skip model: (2k - 1 - 2s) * r_max (rounded up) must not exceed 128");
  } else {
    s = k;
  }
  lv_status st = check_shape(n, s, r_max, mode);
  if (st != LV_OK) return st;
  if (strategy == LV_GENERAL_HYBRID) {
    if (p < 1 || p > kMaxGeneralCols)
      return fail(LV_EINVAL, "p = %lld outside [1, %d] (hybrid deltas)", (long long)p, kMaxGeneralCols);
  } else if (strategy == LV_GENERAL_FACTORED) {
    if (p < 1 || p > kMaxGeneralColsF)
      return fail(LV_EINVAL, "p = %lld outside [1, %d] (factored deltas)", (long long)p, kMaxGeneralColsF);
    if ((int64_t)s * next_pow2(r_max) > kMaxGeneralWidthF)
      return fail(LV_EINVAL, "factored deltas need k * r_max (rounded up to a power of two) <= %d", kMaxGeneralWidthF);
  } else {
    return fail(LV_EINVAL, "unknown strategy %d", strategy);
  }
  return LV_OK;
}

}  // namespace

extern "C" {

size_t lv_view_footprint_general(int64_t n, int k, int r_max, lv_mode mode, int64_t p, int strategy, int s) {
  if (check_general(n, k, r_max, mode, p, strategy, s) != LV_OK) return 0;
  const int sp = s == 0 ? k : s;
  return make_layout(n, sp, r_max, mode, LV_WITH_SUMS, (int)p, strategy == LV_GENERAL_FACTORED, k).total;
}

lv_status lv_view_create_general(const void* A, int64_t n, int64_t lda, int k, int r_max, lv_mode mode,
                                 const void* T0, int64_t ldt, const void* B, int64_t ldb, int64_t p, int strategy,
                                 int s, void* workspace, size_t ws_bytes, void* stream, lv_view** out) {
  g_err[0] = 0;
  if (out) *out = nullptr;
  lv_status st = check_general(n, k, r_max, mode, p, strategy, s);
  if (st != LV_OK) return st;
  if (!T0 || !B) return fail(LV_EINVAL, "T0 or B is NULL");
  if (ldt < p || ldb < p) return fail(LV_EINVAL, "ldt/ldb smaller than p");
  return create_view(A, n, lda, s == 0 ? k : s, r_max, mode, LV_WITH_SUMS, (int)p, strategy == LV_GENERAL_FACTORED,
                     k, T0, ldt, B, ldb, workspace, ws_bytes, stream, out);
}

static lv_status check_update_args(const lv_view* v, const void* U, const void* V, int64_t r,
                                   int64_t ldu, int64_t ldv) {
  if (!v) return fail(LV_EINVAL, "view is NULL");
  if (!U || !V) return fail(LV_EINVAL, "U or V is NULL");
  if (r < 1 || r > v->r_max) return fail(LV_EINVAL, "rank r = %lld outside [1, %d]", (long long)r, v->r_max);
  if (ldu < r || ldv < r) return fail(LV_EINVAL, "ldu/ldv smaller than r");
  return LV_OK;
}

lv_status lv_view_update(lv_view* v, const void* U, const void* V, int64_t r, int64_t ldu,
                         int64_t ldv, void* stream) {
  g_err[0] = 0;
  lv_status st = check_update_args(v, U, V, r, ldu, ldv);
  if (st != LV_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  st = v->mode == LV_FP64
           ? update_one<double>(v, static_cast<const double*>(U), static_cast<const double*>(V), (int)r, ldu, ldv, s)
           : update_one<float>(v, static_cast<const float*>(U), static_cast<const float*>(V), (int)r, ldu, ldv, s);
  if (st != LV_OK) return st;
  v->updates += 1;
  return periodic_drift(v, s);
}

lv_status lv_view_update_batch(lv_view* v, const void* U, const void* V, int64_t r, int64_t count,
                               int64_t ldu, int64_t ldv, int64_t strideU, int64_t strideV,
                               void* stream) {
  g_err[0] = 0;
  if (count < 0) return fail(LV_EINVAL, "count < 0");
  if (count == 0) return v ? LV_OK : fail(LV_EINVAL, "view is NULL");
  lv_status st = check_update_args(v, U, V, r, ldu, ldv);
  if (st != LV_OK) return st;
  if (count > 1 && (strideU < v->n * ldu || strideV < v->n * ldv))
    return fail(LV_EINVAL, "strides smaller than one n x r factor");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (count > 1 && v->pipeline && !v->timing && v->L.pipe_slots > 1)
    return v->mode == LV_FP64
               ? update_batch_pipelined<double>(v, static_cast<const char*>(U), static_cast<const char*>(V), (int)r,
                                                count, ldu, ldv, strideU, strideV, s)
               : update_batch_pipelined<float>(v, static_cast<const char*>(U), static_cast<const char*>(V), (int)r,
                                               count, ldu, ldv, strideU, strideV, s);
  const size_t es = v->L.elem;
  for (int64_t t = 0; t < count; ++t) {
    const char* Ut = static_cast<const char*>(U) + (size_t)(t * strideU) * es;
    const char* Vt = static_cast<const char*>(V) + (size_t)(t * strideV) * es;
    st = v->mode == LV_FP64
             ? update_one<double>(v, reinterpret_cast<const double*>(Ut), reinterpret_cast<const double*>(Vt), (int)r, ldu, ldv, s)
             : update_one<float>(v, reinterpret_cast<const float*>(Ut), reinterpret_cast<const float*>(Vt), (int)r, ldu, ldv, s);
    if (st != LV_OK) return st;
    v->updates += 1;
    st = periodic_drift(v, s);
    if (st != LV_OK) return st;
  }
  return LV_OK;
}

static int power_level(const lv_view* v, int power) {
  if (!v || !is_pow2(power) || power > v->k) return -1;
  return ilog2(power);
}

lv_status lv_view_read(const lv_view* v, int power, void* out, int64_t ldo, void* stream) {
  g_err[0] = 0;
  const int j = power_level(v, power);
  if (j < 0) return fail(LV_EINVAL, "power %d is not stored", power);
  if (!out) return fail(LV_EINVAL, "out is NULL");
  if (ldo < v->n) return fail(LV_EINVAL, "ldo < n");
  const size_t es = v->L.elem;
  const char* src = v->base + v->L.P[j];
  return hip_check(hipMemcpy2DAsync(out, ldo * es, src, v->L.ldp * es, v->n * es, v->n,
                                    hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)),
                   "read");
}

lv_status lv_view_read_sum(const lv_view* v, int index, void* out, int64_t ldo, void* stream) {
  g_err[0] = 0;
  const int j = power_level(v, index);
  if (j < 0) return fail(LV_EINVAL, "sum index %d is not stored", index);
  if (!v->L.sums) return fail(LV_ESTATE, "the view was created without LV_WITH_SUMS");
  if (!out) return fail(LV_EINVAL, "out is NULL");
  if (ldo < v->n) return fail(LV_EINVAL, "ldo < n");
  const size_t es = v->L.elem;
  return hip_check(hipMemcpy2DAsync(out, ldo * es, v->base + v->L.S[j], v->L.ldp * es, v->n * es, v->n,
                                    hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)),
                   "read sum");
}

lv_status lv_view_read_general(const lv_view* v, int index, void* out, int64_t ldo, void* stream) {
  g_err[0] = 0;
  if (!v) return fail(LV_EINVAL, "view is NULL");
  if (!v->L.general) return fail(LV_ESTATE, "the view is not a general-form view");
  // T_1, T_2, T_4, ..., T_s, then (skip model) T_2s, T_3s, ..., T_k
  const int j = power_level(v, index);
  size_t off = 0;
  if (j >= 0) {
    off = v->L.T[j];
  } else if (v->L.nsk > 0 && index > v->k && index <= v->L.kT && index % v->k == 0) {
    off = v->L.Tsk + (size_t)(index / v->k - 2) * v->L.tstride;
  } else {
    return fail(LV_EINVAL, "T index %d is not stored", index);
  }
  if (!out) return fail(LV_EINVAL, "out is NULL");
  if (ldo < v->L.p) return fail(LV_EINVAL, "ldo < p");
  const size_t es = v->L.elem;
  return hip_check(hipMemcpy2DAsync(out, ldo * es, v->base + off, v->L.pp * es, v->L.p * es, v->n,
                                    hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)),
                   "read T");
}

const void* lv_view_data(const lv_view* v, int power, int64_t* ld) {
  const int j = power_level(v, power);
  if (j < 0) return nullptr;
  if (ld) *ld = v->L.ldp;
  return v->base + v->L.P[j];
}

lv_status lv_view_reanchor(lv_view* v, void* stream) {
  g_err[0] = 0;
  if (!v) return fail(LV_EINVAL, "view is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  lv_status st = v->mode == LV_FP64 ? build_chain<double>(v, s) : build_chain<float>(v, s);
  if (st == LV_OK) v->reanchors += 1;
  return st;
}

lv_status lv_view_drift_check(lv_view* v, const void* z, double tau, double* residuals, void* stream) {
  g_err[0] = 0;
  if (!v || !z) return fail(LV_EINVAL, "view or z is NULL");
  if (!(tau >= 0.0)) return fail(LV_EINVAL, "tau must be >= 0");
  if (v->L.m == 0) return LV_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  lv_status st = v->mode == LV_FP64 ? drift_check<double>(v, static_cast<const double*>(z), tau, s)
                                    : drift_check<float>(v, static_cast<const double*>(z), tau, s);
  if (st != LV_OK) return st;
  if (residuals)
    st = hip_check(hipMemcpyAsync(residuals, v->residuals(), sizeof(double) * v->L.m, hipMemcpyDeviceToDevice, s),
                   "copy residuals");
  return st;
}

lv_status lv_view_set_drift_check(lv_view* v, int64_t every, double tau, const void* z, void* stream) {
  g_err[0] = 0;
  if (!v) return fail(LV_EINVAL, "view is NULL");
  if (every < 0) return fail(LV_EINVAL, "every = %lld < 0", (long long)every);
  if (tau != tau) return fail(LV_EINVAL, "tau is NaN");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const lv_status st =
      z ? hip_check(launch_vec_pad(static_cast<const double*>(z), v->n, v->drift_z(), v->L.n_pad, s), "copy z")
        : hip_check(launch_sign_vector(v->drift_z(), v->n, v->L.n_pad, 0x4C494E56494557ull, s), "probe vector");
  if (st != LV_OK) return st;
  v->drift_every = every;
  v->drift_tau = tau >= 0.0 ? tau
                 : v->mode == LV_FP64 ? LV_DRIFT_TAU_FP64
                 : v->mode == LV_FP32 ? LV_DRIFT_TAU_FP32 : LV_DRIFT_TAU_BF16SHADOW;
  return LV_OK;
}

lv_status lv_view_write(lv_view* v, int power, const void* src, int64_t lds, void* stream) {
  g_err[0] = 0;
  const int j = power_level(v, power);
  if (j < 0) return fail(LV_EINVAL, "power %d is not stored", power);
  if (!src) return fail(LV_EINVAL, "src is NULL");
  if (lds < v->n) return fail(LV_EINVAL, "lds < n");
  const size_t es = v->L.elem;
  char* dst = v->base + v->L.P[j];
  hipStream_t s = static_cast<hipStream_t>(stream);
  lv_status st = hip_check(hipMemcpy2DAsync(dst, v->L.ldp * es, src, lds * es, v->n * es, v->n,
                                            hipMemcpyDeviceToDevice, s),
                           "write");
  if (st == LV_OK && v->shadowed() && j < v->L.m)
    st = hip_check(launch_to_bf16(v->P<float>(j), v->shadow(j), v->L.n_pad * v->L.ldp, s), "shadow");
  return st;
}

lv_status lv_view_stats(const lv_view* v, lv_stats* out) {
  if (!v || !out) return fail(LV_EINVAL, "view or out is NULL");
  out->n = v->n;
  out->n_pad = v->L.n_pad;
  out->ld = v->L.ldp;
  out->k = v->k;
  out->levels = v->L.m + 1;
  out->r_max = v->r_max;
  out->mode = (int32_t)v->mode;
  out->updates = v->updates;
  out->reanchors = v->reanchors;
  out->footprint = v->L.total;
  unsigned long long cnt = 0;
  double res[kMaxLevel] = {};
  if (hipMemcpy(&cnt, v->drift_counter(), sizeof(cnt), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(res, v->residuals(), sizeof(double) * (v->L.m > 0 ? v->L.m : 1), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(LV_EDEVICE, "reading drift counters failed");
  out->drift_reanchors = (int64_t)cnt;
  double mx = 0.0;
  for (int j = 0; j < v->L.m; ++j) mx = res[j] > mx || res[j] != res[j] ? res[j] : mx;
  out->last_residual = mx;
  out->drift_checks = v->drift_checks;
  out->drift_every = v->drift_every;
  out->drift_tau = v->drift_tau;
  return LV_OK;
}

lv_status lv_view_tile_rows(const lv_view* v, int level, int* rows) {
  if (!v || !rows) return fail(LV_EINVAL, "view or rows is NULL");
  if (level < 0 || level >= v->L.m) return fail(LV_EINVAL, "level %d has no level pass (levels 0..%d)", level, v->L.m - 1);
  *rows = v->tile_rows[level];
  return LV_OK;
}

lv_status lv_view_set_tile_rows(lv_view* v, int level, int rows) {
  if (!v) return fail(LV_EINVAL, "view is NULL");
  if (level < 0 || level >= v->L.m) return fail(LV_EINVAL, "level %d has no level pass (levels 0..%d)", level, v->L.m - 1);
  if (rows < kMinTileRows || rows > kMaxTileRows || rows % 64 != 0)
    return fail(LV_EINVAL, "tile rows %d not a multiple of 64 in [%d, %d]", rows, kMinTileRows, kMaxTileRows);
  v->tile_rows[level] = rows;
  return LV_OK;
}

lv_status lv_view_autotune(lv_view* v, int pipelined, int64_t trial_updates, void* stream, int* chosen) {
  g_err[0] = 0;
  if (!v) return fail(LV_EINVAL, "view is NULL");
  if (v->L.sums) return fail(LV_ESTATE, "autotune takes views without sums or general form");
  if (trial_updates < 2 || trial_updates > 1000) return fail(LV_EINVAL, "trial_updates %lld not in [2, 1000]",
                                                               (long long)trial_updates);
  if (v->L.m == 0) { if (chosen) *chosen = v->tile_rows[0]; return LV_OK; }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return fail(LV_EDEVICE, "hipEventCreate failed");
  }
  // zero updates: every stored value and the update count stay as they are;
  // no drift check, no timing records
  int saved[kMaxLevel];
  for (int j = 0; j < kMaxLevel; ++j) saved[j] = v->tile_rows[j];
  const int64_t updates = v->updates, every = v->drift_every;
  const bool timing = v->timing, pipe = v->pipeline;
  v->drift_every = 0;
  v->timing = false;
  v->pipeline = pipelined != 0;
  const char* Z = v->base + v->L.zfac;
  const int r = v->L.r_pad;
  auto run = [&](int64_t count) -> lv_status {
    if (v->pipeline && v->L.pipe_slots > 1)
      return v->mode == LV_FP64 ? update_batch_pipelined<double>(v, Z, Z, r, count, r, r, 0, 0, s)
                                : update_batch_pipelined<float>(v, Z, Z, r, count, r, r, 0, 0, s);
    for (int64_t t = 0; t < count; ++t) {
      const lv_status st = v->mode == LV_FP64
                               ? update_one<double>(v, reinterpret_cast<const double*>(Z),
                                                    reinterpret_cast<const double*>(Z), r, r, r, s)
                               : update_one<float>(v, reinterpret_cast<const float*>(Z),
                                                   reinterpret_cast<const float*>(Z), r, r, r, s);
      if (st != LV_OK) return st;
    }
    return LV_OK;
  };
  lv_status st = LV_OK;
  float best = 0.0f;
  int best_rows = saved[0];
  for (int rows = kMinTileRows; rows <= kMaxTileRows && st == LV_OK; rows += 128) {
    for (int j = 0; j < v->L.m; ++j) v->tile_rows[j] = rows;
    st = run(2);
    if (st == LV_OK && hipEventRecord(a, s) != hipSuccess) st = fail(LV_EDEVICE, "hipEventRecord failed");
    if (st == LV_OK) st = run(trial_updates);
    if (st == LV_OK && (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess))
      st = fail(LV_EDEVICE, "timing the trial failed");
    float ms = 0.0f;
    if (st == LV_OK && hipEventElapsedTime(&ms, a, b) != hipSuccess) st = fail(LV_EDEVICE, "hipEventElapsedTime failed");
    if (st == LV_OK && (best == 0.0f || ms < best)) { best = ms; best_rows = rows; }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  v->updates = updates;
  v->drift_every = every;
  v->timing = timing;
  v->pipeline = pipe;
  if (st != LV_OK) {
    for (int j = 0; j < kMaxLevel; ++j) v->tile_rows[j] = saved[j];
    return st;
  }
  for (int j = 0; j < v->L.m; ++j) v->tile_rows[j] = best_rows;
  if (chosen) *chosen = best_rows;
  return LV_OK;
}

lv_status lv_view_set_pipeline(lv_view* v, int enable) {
  g_err[0] = 0;
  if (!v) return fail(LV_EINVAL, "view is NULL");
  v->pipeline = enable != 0;
  return LV_OK;
}

lv_status lv_view_set_timing(lv_view* v, int enable) {
  if (!v) return fail(LV_EINVAL, "view is NULL");
  v->timing = enable != 0;
  return LV_OK;
}

lv_status lv_view_timing(lv_view* v, lv_timing* out) {
  if (!v || !out) return fail(LV_EINVAL, "view or out is NULL");
  std::memset(out, 0, sizeof(*out));
  lv_status st = LV_OK;
  for (auto& p : v->pending) {
    float ms = 0.f;
    if (st == LV_OK) {
      if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess)
        st = fail(LV_EDEVICE, "event timing failed");
    }
    if (p.kind == 0) { out->fused_ms += ms; out->fused_launches += 1; }
    else if (p.kind == 1) { out->tail_ms += ms; out->tail_launches += 1; }
    else { out->top_ms += ms; out->top_launches += 1; }
    v->pool.push_back(p.a);
    v->pool.push_back(p.b);
  }
  v->pending.clear();
  return st;
}

void lv_view_destroy(lv_view* v) {
  if (!v) return;
  for (int q = 1; q < v->pipe_nstages; ++q) (void)hipStreamDestroy(v->pstream[q]);
  for (hipEvent_t e : v->pjoin) if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : v->pfree) if (e) (void)hipEventDestroy(e);
  for (auto& row : v->pready)
    for (hipEvent_t e : row) if (e) (void)hipEventDestroy(e);
  if (v->pfork) (void)hipEventDestroy(v->pfork);
  for (auto& p : v->pending) { v->pool.push_back(p.a); v->pool.push_back(p.b); }
  for (hipEvent_t e : v->pool) (void)hipEventDestroy(e);
  delete v;
}

size_t lv_reeval_footprint(int64_t n, int r_max, lv_mode mode) {
  if (mode != LV_FP64 && mode != LV_FP32) return 0;
  if (n < 1 || n > kMaxOrder || r_max < 0 || r_max > kMaxLevelRank) return 0;
  return reeval_bytes(round_up(n, kPadOrder), (int)next_pow2(r_max < 1 ? 1 : r_max), mode == LV_FP64 ? 8 : 4);
}

lv_status lv_reeval(const void* A, int64_t n, int64_t lda, int k, const void* U, const void* V, int64_t r,
                    int64_t ldu, int64_t ldv, lv_mode mode, void* out, int64_t ldo, void* workspace,
                    size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  if (mode != LV_FP64 && mode != LV_FP32) return fail(LV_EINVAL, "unknown mode %d", (int)mode);
  if (n < 1 || n > kMaxOrder) return fail(LV_EINVAL, "n out of range");
  if (!is_pow2(k) || k > kMaxK) return fail(LV_EINVAL, "k = %d is not a power of two in [1, %d]", k, kMaxK);
  if (r < 0 || r > kMaxLevelRank) return fail(LV_EINVAL, "r out of range");
  if (!A || !out || !workspace) return fail(LV_EINVAL, "NULL pointer");
  if (r > 0 && (!U || !V || ldu < r || ldv < r)) return fail(LV_EINVAL, "bad U/V");
  if (lda < n || ldo < n) return fail(LV_EINVAL, "lda/ldo < n");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(LV_ENOMEM, "workspace misaligned");
  const size_t need = lv_reeval_footprint(n, (int)r, mode);
  if (ws_bytes < need) return fail(LV_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  if (mode == LV_FP64)
    return reeval_impl<double>(static_cast<const double*>(A), n, lda, k, static_cast<const double*>(U),
                               static_cast<const double*>(V), (int)r, ldu, ldv, static_cast<double*>(out), ldo,
                               ws, s);
  return reeval_impl<float>(static_cast<const float*>(A), n, lda, k, static_cast<const float*>(U),
                            static_cast<const float*>(V), (int)r, ldu, ldv, static_cast<float*>(out), ldo, ws,
                            s);
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free update
//
// The factor slabs and per-level partials of lv_powers_update_noalloc live in
// one file-scope device array, `scratch`.  Each GPU holds its own copy until
// the process ends; host code never passes the array's name to a kernel but
// the device address hipGetSymbolAddress returns for the current device,
// looked up once per device on the first call there.  Every byte of it that
// a call reads is written earlier in the same call (slab columns by the
// staging kernel and the tails, partials by the level passes), so nothing
// needs clearing between calls; calls that overlap on one GPU race.
namespace {

constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

lv_status scratch_of_current_device(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_check(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(LV_EDEVICE, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_check(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return LV_OK;
}

}  // namespace

extern "C" {

lv_status lv_powers_update_noalloc(void* const* powers, int64_t n, int64_t ld, int k, lv_mode mode, const void* U,
                                   const void* V, int64_t r, int64_t ldu, int64_t ldv, void* stream) {
  g_err[0] = 0;
  if (mode != LV_FP64 && mode != LV_FP32) return fail(LV_EINVAL, "mode must be LV_FP64 or LV_FP32");
  if (n < kPadOrder || n % kPadOrder != 0 || n > kMaxOrder)
    return fail(LV_EINVAL, "n = %lld is not a positive multiple of %d up to %lld", (long long)n, kPadOrder,
                (long long)kMaxOrder);
  if (r < 1 || r > kMaxLevelRank) return fail(LV_EINVAL, "rank r = %lld outside [1, %d]", (long long)r, kMaxLevelRank);
  lv_status st = check_shape(n, k, (int)r, mode);
  if (st != LV_OK) return st;
  const int elem = mode == LV_FP64 ? 8 : 4;
  if (!powers) return fail(LV_EINVAL, "powers is NULL");
  if (ld < n || (ld * elem) % 16 != 0) return fail(LV_EINVAL, "ld = %lld is below n or not a multiple of 16 bytes",
                                                   (long long)ld);
  const int m = ilog2(k);
  for (int j = 0; j <= m; ++j)
    if (!powers[j] || reinterpret_cast<uintptr_t>(powers[j]) % 16 != 0)
      return fail(LV_EINVAL, "powers[%d] is NULL or not 16-byte aligned", j);
  if (!U || !V) return fail(LV_EINVAL, "U or V is NULL");
  if (ldu < r || ldv < r) return fail(LV_EINVAL, "ldu/ldv smaller than r");
  const Layout L = make_layout(n, k, (int)r, mode, 0, 0, false, 0, true);
  if (L.total > kNoAllocScratchBytes)
    return fail(LV_ENOMEM, "n = %lld, k = %d, r = %lld needs %zu bytes of scratch; the static array holds %zu",
                (long long)n, k, (long long)r, L.total, kNoAllocScratchBytes);
  char* base = nullptr;
  st = scratch_of_current_device(&base);
  if (st != LV_OK) return st;
  // a transient view over the caller's powers and the scratch (host only)
  lv_view v;
  v.n = n; v.k = k; v.r_max = (int)r; v.mode = mode; v.L = L; v.L.ldp = ld;
  v.base = base; v.ws_bytes = kNoAllocScratchBytes; v.updates = 0; v.reanchors = 0;
  for (int j = 0; j < kMaxLevel; ++j) v.tile_rows[j] = L.tile_rows;
  for (int j = 0; j <= m; ++j) v.pext[j] = static_cast<char*>(powers[j]);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return mode == LV_FP64
             ? update_one<double>(&v, static_cast<const double*>(U), static_cast<const double*>(V), (int)r, ldu, ldv, s)
             : update_one<float>(&v, static_cast<const float*>(U), static_cast<const float*>(V), (int)r, ldu, ldv, s);
}

}  // extern "C"
