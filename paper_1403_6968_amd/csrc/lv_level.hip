// Level kernels of the IncrExp update (LINVIEW, App. A exponential model)
// other than the fused pass (lv_fused.hip) and the matrix-core skinny passes
// (lv_skinny.hip): the Gram V_j^T U_j, the tail that reduces the partials and
// assembles the next factors, the rank-R update pass, and small helpers.
//
// For one level j of the exponential model the update needs, with the OLD
// stored power P = A^(2^j) and the level factors U_j, V_j (n x R, R = 2^j r):
//     X = P U_j,   Y = P^T V_j,   G = V_j^T U_j,   P += U_j V_j^T
// and then U_{j+1} = [U_j, X + U_j G], V_{j+1} = [Y, V_j]  (Sec. 4.3, App. A).
// The tail reduces the partials of every tile in a fixed order
// (deterministic, no float atomics).  k_level_update is the update pass (the
// top stored power, and every level whose products ran apart).
//
// Layouts (all row-major):
//   P        n_pad x ldp, zero padding beyond n.
//   slab U   n_pad x W; U_j = columns [0, R).
//   slab V   n_pad x W; V_j = columns [W - R, W)  (callers pass the offset base).
//   partX    [nct][n_pad][R]   (nct = n_pad / TC column tiles)
//   partY    [nrt][n_pad][R]   (nrt row tiles)
//   partG    [ng][R][R] double (ng partials, summed by the tail)
#include "lv_device.h"

namespace lv {
namespace {

// ---------------------------------------------------------------- Gram (ranks > 16)
// Partial V_j^T U_j over one row tile (double accumulation, rows in index
// order): factor rows are staged in LDS 16 at a time; block (rt, pc) covers
// pairs [pc * 256 * PPT, (pc + 1) * 256 * PPT) of the R x R result and thread
// t owns the pairs base + t, base + t + 256, ...
template <typename T, int R>
constexpr int gram_ppt() { return (R * R + 255) / 256 < 16 ? (R * R + 255) / 256 : 16; }

template <typename T, int R>
__device__ __forceinline__ void gram_body(const T* __restrict__ Uj, const T* __restrict__ Vj, const int W,
                                          const int n_pad, const int tile_rows, double* __restrict__ partG,
                                          const int rt, const int pc) {
  constexpr int RS = 16;
  constexpr int PPT = gram_ppt<T, R>();
  const int pbase = pc * 256 * PPT;
  __shared__ T su[RS][R];
  __shared__ T sv[RS][R];
  const int tid = threadIdx.x;
  const int row0 = rt * tile_rows;
  const int nrows = min(tile_rows, n_pad - row0);
  double g[PPT];
#pragma unroll
  for (int e = 0; e < PPT; ++e) g[e] = 0.0;
  for (int i0 = row0; i0 < row0 + nrows; i0 += RS) {
    __syncthreads();
    batched_stage<(RS * R + 255) / 256, 256, T>(
        tid, RS * R, [&](int idx) { return Uj[(int64_t)(i0 + idx / R) * W + idx % R]; },
        [&](int idx, T v) { su[idx / R][idx % R] = v; });
    batched_stage<(RS * R + 255) / 256, 256, T>(
        tid, RS * R, [&](int idx) { return Vj[(int64_t)(i0 + idx / R) * W + idx % R]; },
        [&](int idx, T v) { sv[idx / R][idx % R] = v; });
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PPT; ++e) {
      const int pair = pbase + tid + 256 * e;
      if (pair < R * R) {
        const int a = pair / R, b = pair % R;
#pragma unroll
        for (int rr = 0; rr < RS; ++rr) g[e] = fma((double)sv[rr][a], (double)su[rr][b], g[e]);
      }
    }
  }
#pragma unroll
  for (int e = 0; e < PPT; ++e) {
    const int pair = pbase + tid + 256 * e;
    if (pair < R * R) partG[(int64_t)rt * R * R + pair] = g[e];
  }
}

template <typename T, int R>
__global__ void __launch_bounds__(256) k_gram(const GramDesc<T> d) {
  gram_body<T, R>(d.Uj, d.Vj, d.W, d.n_pad, d.tile_rows, d.partG, blockIdx.x, blockIdx.y);
}

template <typename T, int R>
__global__ void __launch_bounds__(256) k_gram_multi(const GramDesc<T>* __restrict__ ds, int nd) {
  const int v = find_desc(ds, nd, (int)blockIdx.x);
  const GramDesc<T> d = load_desc(ds, v);
  const int local = (int)blockIdx.x - d.block_begin;
  gram_body<T, R>(d.Uj, d.Vj, d.W, d.n_pad, d.tile_rows, d.partG, local % d.nrt, local / d.nrt);
}

// G[idx] = sum over t < ng of G[t * count + idx], in index order, into the
// first partial.
__device__ __forceinline__ void gram_sum_body(double* __restrict__ G, const int ng, const int count, const int blk) {
  const int idx = blk * 256 + (int)threadIdx.x;
  if (idx >= count) return;
  double g = 0.0;
  int t = 0;
  for (; t + 8 <= ng; t += 8) {
    double v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = G[(int64_t)(t + e) * count + idx];
#pragma unroll
    for (int e = 0; e < 8; ++e) g += v[e];
  }
  for (; t < ng; ++t) g += G[(int64_t)t * count + idx];
  G[idx] = g;
}

__global__ void __launch_bounds__(256) k_gram_sum(const GramSumDesc d) { gram_sum_body(d.G, d.ng, d.count, blockIdx.x); }

__global__ void __launch_bounds__(256) k_gram_sum_multi(const GramSumDesc* __restrict__ ds, int nd) {
  const GramSumDesc d = load_desc(ds, find_desc(ds, nd, (int)blockIdx.x));
  gram_sum_body(d.G, d.ng, d.count, (int)blockIdx.x - d.block_begin);
}

// ---------------------------------------------------------------- tail
// Per output (row i, column c): x = sum of the column tiles' partial X and
// y = sum of the row tiles' partial Y, each added in tile order in double
// (loads in batches of 8), ug = sum_d U_j[i][d] G[d][c] in double.
// R < 64: one thread per (row, c), the whole G in LDS.  R >= 64: a block
// covers 64 rows x a 32-column slice and holds only G's slice (R x 32
// doubles), each thread 8 rows of one column.  Same sums in the same order
// either way.
template <typename T>
__device__ __forceinline__ double sum_partials(const T* __restrict__ part, const int64_t stride, const int64_t idx,
                                               const int count) {
  double x = 0.0;
  int t = 0;
  for (; t + 8 <= count; t += 8) {
    T v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = part[(t + e) * stride + idx];
#pragma unroll
    for (int e = 0; e < 8; ++e) x += (double)v[e];
  }
  for (; t < count; ++t) x += (double)part[t * stride + idx];
  return x;
}

template <typename T, int R>
__device__ __forceinline__ void tail_body(const T* __restrict__ partX, const T* __restrict__ partY,
                                          const double* __restrict__ partG, const int nct, const int nrt,
                                          const int ng, const int n_pad, T* slabU, T* slabV, const int W,
                                          const int blk) {
  const T* Ucur = slabU;
  T* Unew = slabU + R;
  T* Vnew = slabV + (W - 2 * R);
  const int tid = threadIdx.x;
  const int64_t strideX = (int64_t)n_pad * R;
  if constexpr (R < kSlicedTailRank) {
    // kTailLanes lanes per output entry (i, c): lane s sums the partials
    // s, s + kTailLanes, ... (and the terms d of U_j G with d = s mod
    // kTailLanes), then a butterfly over the lanes adds the lane sums (every
    // lane ends with the same value: each step adds the same two numbers).
    constexpr int TL = kTailLanes;
    __shared__ double G[R * R];
    for (int idx = tid; idx < R * R; idx += 256) {
      double g = 0.0;
      int t = 0;
      for (; t + 4 <= ng; t += 4) {
        double v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = partG[(int64_t)(t + e) * R * R + idx];
#pragma unroll
        for (int e = 0; e < 4; ++e) g += v[e];
      }
      for (; t < ng; ++t) g += partG[(int64_t)t * R * R + idx];
      G[idx] = g;
    }
    __syncthreads();
    const int64_t pairs = (int64_t)n_pad * R;
    const int64_t idx = (int64_t)blk * (256 / TL) + tid / TL;
    const int sl = tid % TL;
    if (idx >= pairs) return;   // whole lane groups leave together
    const int64_t i = idx / R;
    const int c = (int)(idx % R);
    double x = 0.0, y = 0.0, ug = 0.0;
    for (int t = sl; t < nct; t += TL) x += (double)partX[(int64_t)t * strideX + idx];
    for (int t = sl; t < nrt; t += TL) y += (double)partY[(int64_t)t * strideX + idx];
#pragma unroll
    for (int d = sl; d < R; d += TL) ug = fma((double)Ucur[i * W + d], G[d * R + c], ug);
#pragma unroll
    for (int off = TL / 2; off > 0; off >>= 1) {
      x += __shfl_xor(x, off, TL);
      y += __shfl_xor(y, off, TL);
      ug += __shfl_xor(ug, off, TL);
    }
    if (sl == 0) {
      Unew[i * W + c] = (T)(x + ug);
      Vnew[i * W + c] = (T)y;
    }
  } else {
    // Column slice cs of CW columns: lane column cl = tid % CW, row lane
    // rl = tid / CW; the thread takes rows rl + TPR q (q < Q) of the
    // block's RPB rows, so a wave reads whole 128-byte row segments of
    // every partial and carries Q independent sums.  Each entry sums its
    // partials t = 0, 1, ... and its terms d = 0, 1, ... of U_j G in index
    // order.
    constexpr int CW = R < 32 ? R : 32;
    constexpr int NS = R / CW;
    constexpr int TPR = 256 / CW;
    constexpr int Q = kTailRowsPerThread;
    constexpr int RPB = TPR * Q;
    __shared__ double G[R][CW];
    const int rb = blk / NS, cs = blk % NS;
    const int cl = tid % CW, rl = tid / CW;
    const int c = cs * CW + cl;
    {
      // the G slice: each entry sums its ng partials in order; the loads of
      // all of a thread's entries for one partial are issued together
      constexpr int GE = (R * CW + 255) / 256;
      double g[GE];
#pragma unroll
      for (int e = 0; e < GE; ++e) g[e] = 0.0;
      for (int t = 0; t < ng; ++t) {
        double v[GE];
#pragma unroll
        for (int e = 0; e < GE; ++e) {
          const int idx = tid + 256 * e;
          v[e] = idx < R * CW ? partG[(int64_t)t * R * R + (idx / CW) * R + cs * CW + idx % CW] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < GE; ++e) g[e] += v[e];
      }
#pragma unroll
      for (int e = 0; e < GE; ++e) {
        const int idx = tid + 256 * e;
        if (idx < R * CW) G[idx / CW][idx % CW] = g[e];
      }
    }
    __syncthreads();
    int64_t idx[Q];
    double x[Q], y[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      idx[q] = ((int64_t)rb * RPB + rl + TPR * q) * R + c;
      x[q] = 0.0;
      y[q] = 0.0;
    }
#pragma unroll 2
    for (int t = 0; t < nct; ++t) {
      T v[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) v[q] = partX[(int64_t)t * strideX + idx[q]];
#pragma unroll
      for (int q = 0; q < Q; ++q) x[q] += (double)v[q];
    }
#pragma unroll 2
    for (int t = 0; t < nrt; ++t) {
      T v[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) v[q] = partY[(int64_t)t * strideX + idx[q]];
#pragma unroll
      for (int q = 0; q < Q; ++q) y[q] += (double)v[q];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t i = (int64_t)rb * RPB + rl + TPR * q;
      double ug = 0.0;
#pragma unroll 8
      for (int d = 0; d < R; ++d) ug = fma((double)Ucur[i * W + d], G[d][cl], ug);
      Unew[i * W + c] = (T)(x[q] + ug);
      Vnew[i * W + c] = (T)y[q];
    }
  }
}

template <typename T, int R>
__global__ void __launch_bounds__(256) k_level_tail(const TailDesc<T> d) {
  tail_body<T, R>(d.partX, d.partY, d.partG, d.nct, d.nrt, d.ng, d.n_pad, d.slabU, d.slabV, d.W, blockIdx.x);
}

template <typename T, int R>
__global__ void __launch_bounds__(256) k_level_tail_multi(const TailDesc<T>* __restrict__ ds, int nd) {
  const int v = find_desc(ds, nd, (int)blockIdx.x);
  const TailDesc<T> d = load_desc(ds, v);
  tail_body<T, R>(d.partX, d.partY, d.partG, d.nct, d.nrt, d.ng, d.n_pad, d.slabU, d.slabV, d.W,
                  (int)blockIdx.x - d.block_begin);
}

// ---------------------------------------------------------------- sums tail
// Factors of the sums for the next level (sums of powers, exponential
// model): Q_{j+1} = [U_j, X + Q_j], W_{j+1} = [Y + W_j G, W_j] with
// X = P_j Q_j, Y = S_j^T V_j (partials) and G = Q_j^T V_j (summed).  Q_j
// occupies columns [0, R) of the Q slab and is replaced by U_j in place
// (each thread reads its own entry before writing it); W_j = columns
// [W - R, W) of the W slab.  At level 0 (first): Q_0 = 0, S_0 = I, so
// X = 0, Y = V_0 and W_0 G = 0.
template <typename T, int R>
__device__ __forceinline__ void sums_tail_body(const T* __restrict__ partX, const T* __restrict__ partY,
                                               const double* __restrict__ G, const int nct, const int nrt,
                                               const int n_pad, T* slabQ, T* slabW, const T* __restrict__ Uj,
                                               const T* __restrict__ Vj, const int W, const int first,
                                               const int blk) {
  __shared__ double Gs[R * R];
  const int tid = threadIdx.x;
  if (!first) {
    for (int idx = tid; idx < R * R; idx += 256) Gs[idx] = G[idx];
    __syncthreads();
  }
  const int64_t idx = (int64_t)blk * 256 + tid;
  if (idx >= (int64_t)n_pad * R) return;
  const int64_t i = idx / R;
  const int c = (int)(idx % R);
  const int64_t strideX = (int64_t)n_pad * R;
  double x = 0.0, y, wg = 0.0;
  T q = T(0);
  if (first) {
    y = (double)Vj[i * W + c];
  } else {
    x = sum_partials(partX, strideX, idx, nct);
    y = sum_partials(partY, strideX, idx, nrt);
    const T* Wj = slabW + (W - R);
#pragma unroll
    for (int d = 0; d < R; ++d) wg = fma((double)Wj[i * W + d], Gs[d * R + c], wg);
    q = slabQ[i * W + c];
  }
  slabQ[i * W + R + c] = (T)(x + (double)q);
  slabQ[i * W + c] = Uj[i * W + c];
  slabW[i * W + (W - 2 * R) + c] = (T)(y + wg);
}

template <typename T, int R>
__global__ void __launch_bounds__(256)
k_sums_tail(const T* partX, const T* partY, const double* G, int nct, int nrt, int n_pad, T* slabQ, T* slabW,
            const T* Uj, const T* Vj, int W, int first) {
  sums_tail_body<T, R>(partX, partY, G, nct, nrt, n_pad, slabQ, slabW, Uj, Vj, W, first, blockIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_set_identity(T* __restrict__ S, int64_t ld, int64_t n, int64_t n_pad, const int* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int64_t i = blockIdx.x;
  const int64_t j = (int64_t)blockIdx.y * 256 + threadIdx.x;
  if (j >= n_pad) return;
  S[i * ld + j] = (i == j && i < n) ? T(1) : T(0);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_add(T* __restrict__ dst, const T* __restrict__ src, int64_t count, const int* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) dst[i] += src[i];
}

// ---------------------------------------------------------------- update only
// P += U_j V_j^T.  Lane holds a 16-byte column group (its V_j rows stay in
// registers); the wave walks blocks of 8 rows in the interleaved row slices
// of the fused pass, with the next block's rows of P and U_j requested
// before the current block is updated.  The block's U_j entries come with
// one gathered vector load per 64 entries; the wave stores them to its LDS
// block and reads them back row by row as broadcasts.
// Ranks above 16 are processed in groups of 16 columns of the factors.
// SH (float only): the new values are also written to the bfloat16 shadow S
// (same ld).
template <typename T, int R, bool SH>
__device__ __forceinline__ void update_body(T* __restrict__ P, const int64_t ldp, const int n_pad,
                                            const int tile_rows, const T* __restrict__ Uj,
                                            const T* __restrict__ Vj, const int W, uint16_t* __restrict__ S,
                                            const int ct, const int rt) {
  constexpr int EPL = 16 / (int)sizeof(T);
  constexpr int TC = 64 * EPL;
  constexpr int RG = R < 16 ? R : 16;
  constexpr int NG = R / RG;
  constexpr int RB = 8;
  // U_j entries per lane per block (one factor group; several groups, double
  // storage at ranks above 16, read U_j rows through the scalar unit)
  constexpr int FN = NG == 1 ? (RB * R + 63) / 64 : 1;
  const int lane = threadIdx.x & 63;
  const int wave = wave_id();
  const int col0 = ct * TC;
  const int lc = col0 + lane * EPL;
  // interleaved row slices (as the fused pass): slice rt of ns owns the row
  // blocks rt, rt + ns, rt + 2 ns, ...; wave w every fourth of them from w
  const int ns = (n_pad + tile_rows - 1) / tile_rows;
  const int nb_all = n_pad / RB;

  V16<T> p[RB], pn[RB];
  T fu[FN], fun[FN];
  auto load = [&](int b, V16<T>* pp, T* ff) {
    const int64_t r0 = (int64_t)b * RB;
#pragma unroll
    for (int t = 0; t < RB; ++t) pp[t] = ld16_nt(P + (r0 + t) * ldp + lc);
    if constexpr (NG == 1) {
#pragma unroll
      for (int f = 0; f < FN; ++f) {
        const int e = lane + 64 * f;
        ff[f] = e < RB * R ? Uj[(r0 + e / R) * W + e % R] : T(0);
      }
    }
  };
  T vcol[EPL][NG == 1 ? RG : 1];
  if constexpr (NG == 1) {
#pragma unroll
    for (int q = 0; q < EPL; ++q)
#pragma unroll
      for (int c = 0; c < RG; ++c) vcol[q][c] = Vj[(int64_t)(lc + q) * W + c];
  }

  __shared__ __align__(16) T facs[4][NG == 1 ? RB * R : 1];
  T* fac = facs[wave];

  int b = rt + ns * wave;
  if (b < nb_all) load(b, p, fu);
  for (; b < nb_all; b += 4 * ns) {
    const int64_t r0 = (int64_t)b * RB;
    if constexpr (NG == 1) {
#pragma unroll
      for (int f = 0; f < FN; ++f)
        if (lane + 64 * f < RB * R) fac[lane + 64 * f] = fu[f];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (b + 4 * ns < nb_all) load(b + 4 * ns, pn, fun);
    T d[RB][EPL];
#pragma unroll
    for (int t = 0; t < RB; ++t)
#pragma unroll
      for (int q = 0; q < EPL; ++q) d[t][q] = T(0);
    if constexpr (NG == 1) {
#pragma unroll
      for (int t = 0; t < RB; ++t) {
        T u[RG];
#pragma unroll
        for (int c = 0; c < RG; ++c) u[c] = fac[t * R + c];
#pragma unroll
        for (int q = 0; q < EPL; ++q)
#pragma unroll
          for (int c = 0; c < RG; ++c) d[t][q] = fma(u[c], vcol[q][c], d[t][q]);
      }
    } else {
      for (int g = 0; g < NG; ++g) {
        T vg[EPL][RG];
#pragma unroll
        for (int q = 0; q < EPL; ++q)
#pragma unroll
          for (int c = 0; c < RG; ++c) vg[q][c] = Vj[(int64_t)(lc + q) * W + g * RG + c];
#pragma unroll
        for (int t = 0; t < RB; ++t) {
          const T* urow = Uj + (r0 + t) * W + g * RG;
#pragma unroll
          for (int q = 0; q < EPL; ++q)
#pragma unroll
            for (int c = 0; c < RG; ++c) d[t][q] = fma(urow[c], vg[q][c], d[t][q]);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < RB; ++t) {
#pragma unroll
      for (int q = 0; q < EPL; ++q) p[t].v[q] += d[t][q];
      st16_nt(P + (r0 + t) * ldp + lc, p[t]);
      if constexpr (SH) {
        static_assert(EPL == 4, "shadows are kept for float storage only");
        ushort4 sh;
        sh.x = bf16_rne(p[t].v[0]); sh.y = bf16_rne(p[t].v[1]);
        sh.z = bf16_rne(p[t].v[2]); sh.w = bf16_rne(p[t].v[3]);
        *reinterpret_cast<ushort4*>(S + (r0 + t) * ldp + lc) = sh;
      }
    }
#pragma unroll
    for (int t = 0; t < RB; ++t) p[t] = pn[t];
#pragma unroll
    for (int f = 0; f < FN; ++f) fu[f] = fun[f];
    // the next block's entries overwrite the LDS block only after every
    // lane has read this block's
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

typedef float v16f __attribute__((ext_vector_type(16)));

// P += U_j V_j^T on the matrix cores for float storage and R >= 32
// (v_mfma_f32_32x32x2f32: float products, float accumulation).  Tile
// 128 x 128; wave (wm, wn) owns the 64 x 64 quarter as 2 x 2 blocks of
// 32 x 32.  The tile's factor rows pass through LDS 32 columns at a time.
// In the four steps of a column group, lanes 0-31 supply column c0 + e and
// lanes 32-63 column c0 + 4 + e (e = 0..3) for both U and V, so every
// column of the sum is taken once.  The delta is accumulated from zero and
// added to the old values (requested before the products) once.
// Accumulator element v of lane l is row 8 (v / 4) + 4 (l / 32) + v % 4,
// column l % 32 of its block.
template <int R, bool SH>
__device__ __forceinline__ void update_mfma_body(float* __restrict__ P, const int64_t ldp,
                                                 const float* __restrict__ Uj, const float* __restrict__ Vj,
                                                 const int W, uint16_t* __restrict__ S, const int ct, const int rt) {
  constexpr int TT = kMfmaUpdateTile, KC = 32, KP = KC + 4;
  static_assert(R % KC == 0, "rank must be a multiple of 32");
  __shared__ __align__(16) float sU[TT][KP];
  __shared__ __align__(16) float sV[TT][KP];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = wave_id();
  const int wm = wave >> 1, wn = wave & 1;
  const int l32 = lane & 31, lh = lane >> 5;
  const int row0 = rt * TT, col0 = ct * TT;

  float p[2][2][16];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v)
        p[a][b][v] = __builtin_nontemporal_load(&P[(int64_t)(row0 + wm * 64 + a * 32 + 8 * (v / 4) + 4 * lh +
                                                         (v % 4)) * ldp + col0 + wn * 64 + b * 32 + l32]);
  v16f acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.f;

  for (int kc = 0; kc < R; kc += KC) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TT * KC / 4 / 256; ++i) {
      const int q = tid + 256 * i;
      const int r = q >> 3, c4 = (q & 7) * 4;
      *reinterpret_cast<float4*>(&sU[r][c4]) = *reinterpret_cast<const float4*>(Uj + (int64_t)(row0 + r) * W + kc + c4);
      *reinterpret_cast<float4*>(&sV[r][c4]) = *reinterpret_cast<const float4*>(Vj + (int64_t)(col0 + r) * W + kc + c4);
    }
    __syncthreads();
#pragma unroll
    for (int c0 = 0; c0 < KC; c0 += 8) {
      float4 ua[2], vb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) ua[a] = *reinterpret_cast<const float4*>(&sU[wm * 64 + a * 32 + l32][c0 + 4 * lh]);
#pragma unroll
      for (int b = 0; b < 2; ++b) vb[b] = *reinterpret_cast<const float4*>(&sV[wn * 64 + b * 32 + l32][c0 + 4 * lh]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ua[a].x, vb[b].x, acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ua[a].y, vb[b].y, acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ua[a].z, vb[b].z, acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(ua[a].w, vb[b].w, acc[a][b], 0, 0, 0);
        }
    }
  }

#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t o = (int64_t)(row0 + wm * 64 + a * 32 + 8 * (v / 4) + 4 * lh + (v % 4)) * ldp + col0 +
                          wn * 64 + b * 32 + l32;
        const float x = p[a][b][v] + acc[a][b][v];
        __builtin_nontemporal_store(x, &P[o]);
        if constexpr (SH) S[o] = bf16_rne(x);
      }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float bf16_value(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

// P += U_j V_j^T in the bfloat16-shadow mode for R >= 32, on the bfloat16
// matrix cores with split operands: x = hi + lo with hi = bf16(x) and
// lo = bf16(x - hi), and u v ~ hi_u hi_v + hi_u lo_v + lo_u hi_v (three
// v_mfma_f32_32x32x16_bf16, float accumulation).  The dropped lo_u lo_v and
// the rounding of lo leave a relative error of about 2^-16 per product.
// Same tiles, waves and accumulator layout as update_mfma_body; a lane of a
// 16-column step supplies factor columns 8 (l / 32) + e, e = 0..7, for both
// operands.
template <int R, bool SH>
__device__ __forceinline__ void update_split_body(float* __restrict__ P, const int64_t ldp,
                                                  const float* __restrict__ Uj, const float* __restrict__ Vj,
                                                  const int W, uint16_t* __restrict__ S, const int ct, const int rt) {
  constexpr int TT = kMfmaUpdateTile, KC = 32, KP = KC + 8;
  static_assert(R % KC == 0, "rank must be a multiple of 32");
  __shared__ __align__(16) uint16_t sUh[TT][KP], sUl[TT][KP], sVh[TT][KP], sVl[TT][KP];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = wave_id();
  const int wm = wave >> 1, wn = wave & 1;
  const int l32 = lane & 31, lh = lane >> 5;
  const int row0 = rt * TT, col0 = ct * TT;

  // The old values: requested before the products (their loads overlap the
  // products); from R = 128 after them, so that the products run without
  // the 64 registers they occupy (two waves per SIMD instead of one then
  // hide the latency; see update_min_waves)
  constexpr bool LATE_P = R >= 128;
  float p[2][2][16];
  auto load_p = [&]() {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v)
          p[a][b][v] = __builtin_nontemporal_load(&P[(int64_t)(row0 + wm * 64 + a * 32 + 8 * (v / 4) + 4 * lh +
                                                           (v % 4)) * ldp + col0 + wn * 64 + b * 32 + l32]);
  };
  if constexpr (!LATE_P) load_p();
  v16f acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[a][b][v] = 0.f;

  // The factor values of the next column group are requested before the
  // products of the current one (registers: 8 float4 per thread).
  constexpr int SPT = TT * KC / 4 / 256;
  float4 nu[SPT], nw[SPT];
  auto fetch_uv = [&](const int kc) {
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
      const int q = tid + 256 * i;
      const int r = q >> 3, c4 = (q & 7) * 4;
      nu[i] = *reinterpret_cast<const float4*>(Uj + (int64_t)(row0 + r) * W + kc + c4);
      nw[i] = *reinterpret_cast<const float4*>(Vj + (int64_t)(col0 + r) * W + kc + c4);
    }
  };
  fetch_uv(0);
  for (int kc = 0; kc < R; kc += KC) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SPT; ++i) {
      const int q = tid + 256 * i;
      const int r = q >> 3, c4 = (q & 7) * 4;
      const float4 u = nu[i], w = nw[i];
      const float uu[4] = {u.x, u.y, u.z, u.w}, ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint16_t uh = bf16_rne(uu[e]), wh = bf16_rne(ww[e]);
        sUh[r][c4 + e] = uh;
        sUl[r][c4 + e] = bf16_rne(uu[e] - bf16_value(uh));
        sVh[r][c4 + e] = wh;
        sVl[r][c4 + e] = bf16_rne(ww[e] - bf16_value(wh));
      }
    }
    __syncthreads();
    if (kc + KC < R) fetch_uv(kc + KC);
#pragma unroll
    for (int ks = 0; ks < KC; ks += 16) {
      bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        ah[a] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&sUh[wm * 64 + a * 32 + l32][ks + 8 * lh]));
        al[a] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&sUl[wm * 64 + a * 32 + l32][ks + 8 * lh]));
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        bh[b] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&sVh[wn * 64 + b * 32 + l32][ks + 8 * lh]));
        bl[b] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&sVl[wn * 64 + b * 32 + l32][ks + 8 * lh]));
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
        }
    }
  }

  if constexpr (LATE_P) load_p();
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t o = (int64_t)(row0 + wm * 64 + a * 32 + 8 * (v / 4) + 4 * lh + (v % 4)) * ldp + col0 +
                          wn * 64 + b * 32 + l32;
        const float x = p[a][b][v] + acc[a][b][v];
        __builtin_nontemporal_store(x, &P[o]);
        if constexpr (SH) S[o] = bf16_rne(x);
      }
}

// SPLIT selects the split-bfloat16 products (bfloat16-shadow mode) for the
// matrix-core ranks.
template <typename T, int R, bool SH, bool SPLIT>
__device__ __forceinline__ void update_any(const UpdateDesc<T>& d, const int ct, const int rt) {
  if constexpr (sizeof(T) == 4 && R >= kMfmaUpdateRank && SPLIT)
    update_split_body<R, SH>(d.P, d.ldp, d.Uj, d.Vj, d.W, d.S, ct, rt);
  else if constexpr (sizeof(T) == 4 && R >= kMfmaUpdateRank)
    update_mfma_body<R, SH>(d.P, d.ldp, d.Uj, d.Vj, d.W, d.S, ct, rt);
  else
    update_body<T, R, SH>(d.P, d.ldp, d.n_pad, d.tile_rows, d.Uj, d.Vj, d.W, d.S, ct, rt);
}

// Float matrix-core ranks: at least two waves per SIMD (the 128 x 128
// tile's old values stay in registers while its delta is formed).  The
// split-bfloat16 products from R = 128 too, where the old values are loaded
// after the products; below, their unrolled chunks fit without a bound.
template <typename T, int R, bool SPLIT> constexpr int update_min_waves() {
  return sizeof(T) == 4 && R >= kMfmaUpdateRank && (!SPLIT || R >= 128) ? 2 : 1;
}

template <typename T, int R, bool SH, bool SPLIT>
__global__ void __launch_bounds__(256, (update_min_waves<T, R, SPLIT>())) k_level_update(const UpdateDesc<T> d) {
  update_any<T, R, SH, SPLIT>(d, blockIdx.x, blockIdx.y);
}

template <typename T, int R, bool SH, bool SPLIT>
__global__ void __launch_bounds__(256, (update_min_waves<T, R, SPLIT>()))
k_level_update_multi(const UpdateDesc<T>* __restrict__ ds, int nd) {
  const int v = find_desc(ds, nd, (int)blockIdx.x);
  const UpdateDesc<T> d = load_desc(ds, v);
  const int local = (int)blockIdx.x - d.block_begin;
  update_any<T, R, SH, SPLIT>(d, local % d.nct, local / d.nct);
}

// ---------------------------------------------------------------- small kernels
template <typename Tin, typename Tout>
__global__ void __launch_bounds__(256)
k_copy_pad(const Tin* __restrict__ src, int64_t lds, int64_t n, Tout* __restrict__ dst,
           int64_t ldd, int64_t n_pad, const int* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int64_t i = blockIdx.x;
  const int64_t j = (int64_t)blockIdx.y * 256 + threadIdx.x;
  if (j >= n_pad) return;
  const Tout v = (i < n && j < n) ? (Tout)src[i * lds + j] : Tout(0);
  dst[i * ldd + j] = v;
}

template <typename T>
__device__ __forceinline__ void prep_body(const T* __restrict__ U, const int64_t ldu, const T* __restrict__ V,
                                          const int64_t ldv, const int64_t n, const int r, const int r_pad,
                                          T* __restrict__ slabU, T* __restrict__ slabV, const int W,
                                          const int64_t n_pad, const int blk) {
  const int64_t idx = (int64_t)blk * 256 + threadIdx.x;
  if (idx >= n_pad * r_pad) return;
  const int64_t i = idx / r_pad;
  const int c = (int)(idx % r_pad);
  const bool in = i < n && c < r;
  slabU[i * W + c] = in ? U[i * ldu + c] : T(0);
  slabV[i * W + (W - r_pad) + c] = in ? V[i * ldv + c] : T(0);
}

template <typename T>
__global__ void __launch_bounds__(256) k_prep(const PrepDesc<T> d) {
  prep_body<T>(d.U, d.ldu, d.V, d.ldv, d.n, d.r, d.r_pad, d.slabU, d.slabV, d.W, d.n_pad, blockIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(256) k_prep_multi(const PrepDesc<T>* __restrict__ ds, int nd) {
  const int v = find_desc(ds, nd, (int)blockIdx.x);
  const PrepDesc<T> d = load_desc(ds, v);
  prep_body<T>(d.U, d.ldu, d.V, d.ldv, d.n, d.r, d.r_pad, d.slabU, d.slabV, d.W, d.n_pad,
               (int)blockIdx.x - d.block_begin);
}

template <typename T, int R>
hipError_t update_r(T* P, int64_t ldp, int64_t n_pad, const T* Uj, const T* Vj, int W,
                    hipStream_t s, uint16_t* S, bool split) {
  const int tile_rows = update_slice_rows(R, (int)sizeof(T), n_pad);
  const int nct = (int)(n_pad / update_tile_cols(R, (int)sizeof(T)));
  const UpdateDesc<T> d{P, ldp, (int)n_pad, tile_rows, Uj, Vj, W, nct, 0, S};
  const dim3 grid((unsigned)nct, (unsigned)((n_pad + tile_rows - 1) / tile_rows));
  if constexpr (sizeof(T) == 4) {
    if (S != nullptr && split)
      hipLaunchKernelGGL((k_level_update<T, R, true, true>), grid, dim3(256), 0, s, d);
    else if (S != nullptr)
      hipLaunchKernelGGL((k_level_update<T, R, true, false>), grid, dim3(256), 0, s, d);
    else if (split)
      hipLaunchKernelGGL((k_level_update<T, R, false, true>), grid, dim3(256), 0, s, d);
    else
      hipLaunchKernelGGL((k_level_update<T, R, false, false>), grid, dim3(256), 0, s, d);
    return hipGetLastError();
  }
  if (S != nullptr || split) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_level_update<T, R, false, false>), grid, dim3(256), 0, s, d);
  return hipGetLastError();
}

// Stand-alone Gram: gram_tiles(n_pad) partials, then their sum into the first.
template <typename T, int R>
hipError_t gram_r(const T* Uj, const T* Vj, int W, int64_t n_pad, double* partG, hipStream_t s) {
  const int ng = gram_tiles(n_pad);
  const GramDesc<T> g{Uj, Vj, W, (int)n_pad, kGramRows, partG, ng, 0};
  const dim3 ggrid((unsigned)ng, (unsigned)((R * R + gram_pairs_per_block(R) - 1) / gram_pairs_per_block(R)));
  hipLaunchKernelGGL((k_gram<T, R>), ggrid, dim3(256), 0, s, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const GramSumDesc gs{partG, ng, R * R, 0};
  hipLaunchKernelGGL(k_gram_sum, dim3((unsigned)((R * R + 255) / 256)), dim3(256), 0, s, gs);
  return hipGetLastError();
}

template <typename T, int R>
hipError_t tail_r(const T* partX, const T* partY, const double* partG, int nct, int nrt, int ng,
                  int64_t n_pad, T* slabU, T* slabV, int W, hipStream_t s) {
  const TailDesc<T> d{partX, partY, partG, nct, nrt, (int)n_pad, slabU, slabV, W, 0, ng};
  hipLaunchKernelGGL((k_level_tail<T, R>), dim3((unsigned)tail_blocks(n_pad, R)), dim3(256), 0, s, d);
  return hipGetLastError();
}

}  // namespace

template <typename Tin, typename Tout>
hipError_t launch_copy_pad(const Tin* src, int64_t lds, int64_t n, Tout* dst, int64_t ldd,
                           int64_t n_pad, hipStream_t s, const int* gate) {
  const dim3 grid((unsigned)n_pad, (unsigned)((n_pad + 255) / 256));
  hipLaunchKernelGGL((k_copy_pad<Tin, Tout>), grid, dim3(256), 0, s, src, lds, n, dst, ldd, n_pad, gate);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prep(const T* U, int64_t ldu, const T* V, int64_t ldv, int64_t n, int r,
                       int r_pad, T* slabU, T* slabV, int W, int64_t n_pad, hipStream_t s) {
  const PrepDesc<T> d{U, ldu, V, ldv, n, r, r_pad, slabU, slabV, W, n_pad, 0};
  hipLaunchKernelGGL((k_prep<T>), dim3((unsigned)((n_pad * r_pad + 255) / 256)), dim3(256), 0, s, d);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_level_tail(int R, const T* partX, const T* partY, const double* partG, int nct,
                             int nrt, int ng, int64_t n_pad, T* slabU, T* slabV, int W, hipStream_t s) {
  if (R == kMaxLevelRank) return tail_r<T, kMaxLevelRank>(partX, partY, partG, nct, nrt, ng, n_pad, slabU, slabV, W, s);
  LV_RANK_SWITCH(R, return (tail_r<T, RR>(partX, partY, partG, nct, nrt, ng, n_pad, slabU, slabV, W, s)))
}

template <typename T>
hipError_t launch_level_update(int R, T* P, int64_t ldp, int64_t n_pad, const T* slabU,
                               const T* slabV, int W, hipStream_t s, uint16_t* S, bool split) {
  const T* Uj = slabU;
  const T* Vj = slabV + (W - R);
  if (R == 2 * kMaxLevelRank) return update_r<T, 2 * kMaxLevelRank>(P, ldp, n_pad, Uj, Vj, W, s, S, split);
  if (R == kMaxLevelRank) return update_r<T, kMaxLevelRank>(P, ldp, n_pad, Uj, Vj, W, s, S, split);
  LV_RANK_SWITCH(R, return (update_r<T, RR>(P, ldp, n_pad, Uj, Vj, W, s, S, split)))
}

template <typename T>
hipError_t launch_level_gram(int R, const T* slabU, const T* slabV, int W, int64_t n_pad, double* partG,
                             hipStream_t s) {
  const T* Uj = slabU;
  const T* Vj = slabV + (W - R);
  if (R == kMaxLevelRank) return gram_r<T, kMaxLevelRank>(Uj, Vj, W, n_pad, partG, s);
  LV_RANK_SWITCH(R, return (gram_r<T, RR>(Uj, Vj, W, n_pad, partG, s)))
}

template <typename T>
hipError_t launch_gram_multi(int R, const GramDesc<T>* ds, int nd, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (R == kMaxLevelRank) {
    hipLaunchKernelGGL((k_gram_multi<T, kMaxLevelRank>), dim3((unsigned)blocks), dim3(256), 0, s, ds, nd);
    return hipGetLastError();
  }
  LV_RANK_SWITCH(R, hipLaunchKernelGGL((k_gram_multi<T, RR>), dim3((unsigned)blocks), dim3(256), 0, s, ds, nd);
                 return hipGetLastError())
}

template <typename T>
hipError_t launch_gram_cols(int R, const T* Uop, const T* Vop, int W, int64_t n_pad, double* partG, hipStream_t s) {
  LV_RANK_SWITCH(R, return (gram_r<T, RR>(Uop, Vop, W, n_pad, partG, s)))
}

template <typename T>
hipError_t launch_sums_tail(int R, const T* partX, const T* partY, const double* G, int nct, int nrt, int64_t n_pad,
                            T* slabQ, T* slabW, const T* slabU, const T* slabV, int W, bool first, hipStream_t s) {
  const T* Uj = slabU;
  const T* Vj = slabV + (W - R);
  const dim3 grid((unsigned)((n_pad * R + 255) / 256));
  LV_RANK_SWITCH(R, hipLaunchKernelGGL((k_sums_tail<T, RR>), grid, dim3(256), 0, s, partX, partY, G, nct, nrt,
                                       (int)n_pad, slabQ, slabW, Uj, Vj, W, first ? 1 : 0);
                 return hipGetLastError())
}

template <typename T>
hipError_t launch_set_identity(T* S, int64_t ld, int64_t n, int64_t n_pad, hipStream_t s, const int* gate) {
  hipLaunchKernelGGL((k_set_identity<T>), dim3((unsigned)n_pad, (unsigned)((n_pad + 255) / 256)), dim3(256), 0, s, S,
                     ld, n, n_pad, gate);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_add(T* dst, const T* src, int64_t count, hipStream_t s, const int* gate) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_add<T>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, dst, src, count, gate);
  return hipGetLastError();
}

hipError_t launch_gram_sum(double* G, int ng, int count, hipStream_t s) {
  const GramSumDesc d{G, ng, count, 0};
  hipLaunchKernelGGL(k_gram_sum, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_gram_sum_multi(const GramSumDesc* ds, int nd, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gram_sum_multi, dim3((unsigned)blocks), dim3(256), 0, s, ds, nd);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tail_multi(int R, const TailDesc<T>* ds, int nd, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (R == kMaxLevelRank) {
    hipLaunchKernelGGL((k_level_tail_multi<T, kMaxLevelRank>), dim3((unsigned)blocks), dim3(256), 0, s, ds, nd);
    return hipGetLastError();
  }
  LV_RANK_SWITCH(R, hipLaunchKernelGGL((k_level_tail_multi<T, RR>), dim3((unsigned)blocks), dim3(256), 0, s, ds, nd);
                 return hipGetLastError())
}

template <typename T, bool SH, bool SPLIT>
hipError_t update_multi_sh(int R, const UpdateDesc<T>* ds, int nd, int blocks, hipStream_t s) {
  if (R == 2 * kMaxLevelRank) {
    hipLaunchKernelGGL((k_level_update_multi<T, 2 * kMaxLevelRank, SH, SPLIT>), dim3((unsigned)blocks), dim3(256), 0, s,
                       ds, nd);
    return hipGetLastError();
  }
  if (R == kMaxLevelRank) {
    hipLaunchKernelGGL((k_level_update_multi<T, kMaxLevelRank, SH, SPLIT>), dim3((unsigned)blocks), dim3(256), 0, s,
                       ds, nd);
    return hipGetLastError();
  }
  LV_RANK_SWITCH(R, hipLaunchKernelGGL((k_level_update_multi<T, RR, SH, SPLIT>), dim3((unsigned)blocks), dim3(256), 0,
                                       s, ds, nd);
                 return hipGetLastError())
}

template <typename T>
hipError_t launch_update_multi(int R, bool shadow, bool split, const UpdateDesc<T>* ds, int nd, int blocks,
                               hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if constexpr (sizeof(T) == 4) {
    if (shadow && split) return update_multi_sh<T, true, true>(R, ds, nd, blocks, s);
    if (shadow) return update_multi_sh<T, true, false>(R, ds, nd, blocks, s);
    if (split) return update_multi_sh<T, false, true>(R, ds, nd, blocks, s);
    return update_multi_sh<T, false, false>(R, ds, nd, blocks, s);
  }
  if (shadow || split) return hipErrorInvalidValue;
  return update_multi_sh<T, false, false>(R, ds, nd, blocks, s);
}

template <typename T>
hipError_t launch_prep_multi(const PrepDesc<T>* ds, int nd, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_prep_multi<T>), dim3((unsigned)blocks), dim3(256), 0, s, ds, nd);
  return hipGetLastError();
}

#define LV_INST(T)                                                                              \
  template hipError_t launch_prep<T>(const T*, int64_t, const T*, int64_t, int64_t, int, int,     \
                                     T*, T*, int, int64_t, hipStream_t);                          \
  template hipError_t launch_level_tail<T>(int, const T*, const T*, const double*, int, int, int, \
                                           int64_t, T*, T*, int, hipStream_t);                    \
  template hipError_t launch_level_update<T>(int, T*, int64_t, int64_t, const T*, const T*, int,  \
                                             hipStream_t, uint16_t*, bool);                       \
  template hipError_t launch_level_gram<T>(int, const T*, const T*, int, int64_t, double*,        \
                                           hipStream_t);                                          \
  template hipError_t launch_gram_multi<T>(int, const GramDesc<T>*, int, int, hipStream_t);        \
  template hipError_t launch_tail_multi<T>(int, const TailDesc<T>*, int, int, hipStream_t);        \
  template hipError_t launch_update_multi<T>(int, bool, bool, const UpdateDesc<T>*, int, int, hipStream_t); \
  template hipError_t launch_prep_multi<T>(const PrepDesc<T>*, int, int, hipStream_t);                    \
  template hipError_t launch_gram_cols<T>(int, const T*, const T*, int, int64_t, double*, hipStream_t);    \
  template hipError_t launch_sums_tail<T>(int, const T*, const T*, const double*, int, int, int64_t, T*, T*, \
                                          const T*, const T*, int, bool, hipStream_t);                     \
  template hipError_t launch_set_identity<T>(T*, int64_t, int64_t, int64_t, hipStream_t, const int*);      \
  template hipError_t launch_add<T>(T*, const T*, int64_t, hipStream_t, const int*);
LV_INST(float)
LV_INST(double)
#undef LV_INST

template hipError_t launch_copy_pad<float, float>(const float*, int64_t, int64_t, float*, int64_t, int64_t, hipStream_t, const int*);
template hipError_t launch_copy_pad<double, double>(const double*, int64_t, int64_t, double*, int64_t, int64_t, hipStream_t, const int*);
template hipError_t launch_copy_pad<float, double>(const float*, int64_t, int64_t, double*, int64_t, int64_t, hipStream_t, const int*);
template hipError_t launch_copy_pad<double, float>(const double*, int64_t, int64_t, float*, int64_t, int64_t, hipStream_t, const int*);

}  // namespace lv
