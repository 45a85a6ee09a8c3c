// Read-only skinny-product passes of a level on the matrix cores (App. A,
// with the OLD power P_j):  X = P_j U_j,  Y^T = V_j^T P_j.
//
// BF16-shadow form (storage FP32): every stored power below the top keeps a
// bfloat16 copy S_j, rewritten by the update pass that adds U_j V_j^T to
// P_j.  k_skinny_bf16 reads the shadow (2 bytes per element) and multiplies
// bfloat16 x bfloat16 with float accumulation (v_mfma_f32_32x32x16_bf16).
// k_skinny_f32 reads the float power itself and multiplies in float
// (v_mfma_f32_32x32x2f32): the FP32 method's products at level ranks where
// the vector units, not HBM, would bound a fused pass; k_skinny16_f32 is
// its 16-column form (v_mfma_f32_16x16x4f32), and k_xprod_f32 forms X alone
// with P loaded straight into the operand registers (no LDS staging).
// All write the partial X / Y layouts of the fused pass, so the common tail
// assembles the next factors; the Gram V_j^T U_j is formed in FP64 apart.
//
// Lane layouts (64 lanes, l = lane, h = l / 32):
//   bf16 32x32x16  A: lane l holds A[l % 32][8 h + e], e = 0..7
//                  B: lane l holds B[8 h + e][l % 32]
//   f32 32x32x2    A: lane l holds A[l % 32][h];  B: B[h][l % 32]
//   both           C: element v of lane l is C[8 (v / 4) + 4 h + v % 4][l % 32]
#include "lv_device.h"

#include <type_traits>

namespace lv {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TCB = 256;   // tile columns
constexpr int CRB = 64;    // rows per LDS chunk
constexpr int SPAD = 8;    // LDS row padding (bf16 elements, keeps 16-byte alignment)

// Compile-time loop: f(std::integral_constant<int, I>) for I = 0 .. N-1, so
// that arrays indexed by I stay in registers.
template <int I, int N, typename F> __device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

__device__ __forceinline__ bf16x8 lds8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(p));
}

// Factor entries past column R are the zero padding of the factor blocks.
// Their loads still take place, at column min(c, R - 1), which the row holds:
// a load under a condition becomes a branch of its own, after which the
// compiler waits for it alone, so a run of guarded loads would be served one
// round trip at a time.  fac_clamped is the raw load (prefetches zero the
// padding when they are staged, so that no wait follows the load), and
// fac_or_zero the padded entry.
__device__ __forceinline__ float fac_clamped(const float* __restrict__ row, const int c, const int R) {
  return row[c < R ? c : R - 1];
}
__device__ __forceinline__ float fac_or_zero(const float* __restrict__ row, const int c, const int R) {
  const float v = fac_clamped(row, c, R);
  return c < R ? v : 0.f;
}

// Tile: about tile_rows x 256 columns of S (the slices of a column tile
// interleave by 64-row chunks), walked in chunks through LDS; the next
// chunk or two of S and of V_j are held in registers while the current one
// is used.
// Factor columns are padded with zeros to 32 NB.
//   X: per chunk, the 2 NB (row half, factor block) 32 x 32 outputs are
//      shared round-robin by the 4 waves, K = the tile's 256 columns; one
//      partial per (row, column tile).
//   Y: wave w keeps the accumulators of tile columns [64 w, 64 w + 64) for
//      every factor block over all chunks of the tile (K = rows); one
//      partial per (column, row tile).
// The B operand of Y needs 8 consecutive rows of one column: 8 LDS reads.
template <int NB>
__device__ __forceinline__ void skinny_body(const uint16_t* __restrict__ S, const int64_t ldp, const int n_pad,
                                            const int tile_rows, const float* __restrict__ Uj,
                                            const float* __restrict__ Vj, const int W, const int R,
                                            float* __restrict__ partX, float* __restrict__ partY, const int pR,
                                            const int ct, const int rt) {
  constexpr int RP = 32 * NB;
  __shared__ __align__(16) uint16_t sS[CRB][TCB + SPAD];
  __shared__ __align__(16) uint16_t sUt[RP][TCB + SPAD];
  __shared__ __align__(16) uint16_t sVt[RP][CRB + SPAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col0 = ct * TCB;
  // interleaved chunks: slice rt of ns takes chunks rt, rt + ns, ... (CS
  // rows apart), so the grid streams one band of rows at a time
  const int ns = (n_pad + tile_rows - 1) / tile_rows;
  const int CS = ns * CRB;
  const int row0 = rt * CRB;
  const int rend = n_pad;
  const int l32 = lane % 32, lh = lane / 32;
  // chunk staging: thread -> rows tid / 32 + 8 i, 16-byte column group tid % 32
  const int srow = tid / 32, sgrp = tid % 32;

  constexpr int VPT = RP * CRB / 256;   // V_j values staged per thread and chunk
  // NB = 1: two chunks in flight, buffers A and B alternating (a tile may
  // have an odd number of chunks: tile_rows is any multiple of 64 and the
  // last tile may be ragged, so the second chunk of a pair and its fetch are
  // guarded); larger NB: one chunk (the accumulators need the registers)
  constexpr int DEPTH = NB == 1 ? 2 : 1;
  u16x8 preA[CRB / 8], preB[CRB / 8];
  float pvA[VPT], pvB[VPT];
  auto fetch = [&](u16x8 (&pre)[CRB / 8], float (&pv)[VPT], const int r0) {
#pragma unroll
    for (int i = 0; i < CRB / 8; ++i)
      pre[i] = __builtin_nontemporal_load(reinterpret_cast<const u16x8*>(S + (int64_t)(r0 + srow + 8 * i) * ldp + col0 +
                                                                     sgrp * 8));
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int idx = tid + 256 * i;
      const int rr = idx / RP, c = idx % RP;
      pv[i] = fac_clamped(Vj + (int64_t)(r0 + rr) * W, c, R);
    }
  };
  fetch(preA, pvA, row0);
  if constexpr (DEPTH == 2) {
    if (row0 + CS < rend) fetch(preB, pvB, row0 + CS);
  }

  // U_j rows of the tile's columns, transposed: sUt[c][k] = U_j[col0 + k][c]
  batched_stage<RP * TCB / 256, 256, float>(
      tid, RP * TCB, [&](int idx) { const int c = idx % RP; return fac_or_zero(Uj + (int64_t)(col0 + idx / RP) * W, c, R); },
      [&](int idx, float v) { sUt[idx % RP][idx / RP] = bf16_rne(v); });

  v16f yacc[NB][2];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) yacc[a][b][v] = 0.f;

  auto chunk = [&](u16x8 (&pre)[CRB / 8], float (&pv)[VPT], const int cr0) {
    __syncthreads();   // the previous chunk is no longer read
#pragma unroll
    for (int i = 0; i < CRB / 8; ++i) *reinterpret_cast<u16x8*>(&sS[srow + 8 * i][sgrp * 8]) = pre[i];
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int idx = tid + 256 * i;
      sVt[idx % RP][idx / RP] = bf16_rne(idx % RP < R ? pv[i] : 0.f);
    }
    __syncthreads();
    if (cr0 + DEPTH * CS < rend) fetch(pre, pv, cr0 + DEPTH * CS);

    // X rows of the chunk
    for (int t = wave; t < 2 * NB; t += 4) {
      const int mb = t % 2, nb = t / 2;
      v16f acc;
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[v] = 0.f;
#pragma unroll 4
      for (int ks = 0; ks < TCB / 16; ++ks)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lds8(&sS[mb * 32 + l32][ks * 16 + 8 * lh]),
                                                       lds8(&sUt[nb * 32 + l32][ks * 16 + 8 * lh]), acc, 0, 0, 0);
      const int c = nb * 32 + l32;
      if (c < R) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int rr = mb * 32 + 8 * (v / 4) + 4 * lh + (v % 4);
          partX[((int64_t)ct * n_pad + cr0 + rr) * pR + c] = acc[v];
        }
      }
    }

    // Y^T += V_chunk^T S_chunk
#pragma unroll
    for (int ks = 0; ks < CRB / 16; ++ks) {
#pragma unroll
      for (int cbi = 0; cbi < 2; ++cbi) {
        const int colc = (2 * wave + cbi) * 32 + l32;
        u16x8 bv;
#pragma unroll
        for (int e = 0; e < 8; ++e) bv[e] = sS[ks * 16 + 8 * lh + e][colc];
        const bf16x8 b = __builtin_bit_cast(bf16x8, bv);
#pragma unroll
        for (int nbr = 0; nbr < NB; ++nbr)
          yacc[nbr][cbi] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(lds8(&sVt[nbr * 32 + l32][ks * 16 + 8 * lh]), b,
                                                                   yacc[nbr][cbi], 0, 0, 0);
      }
    }
  };

  if constexpr (DEPTH == 2) {
    for (int cr0 = row0; cr0 < rend; cr0 += 2 * CS) {
      chunk(preA, pvA, cr0);
      if (cr0 + CS < rend) chunk(preB, pvB, cr0 + CS);
    }
  } else {
    for (int cr0 = row0; cr0 < rend; cr0 += CS) chunk(preA, pvA, cr0);
  }

#pragma unroll
  for (int nbr = 0; nbr < NB; ++nbr)
#pragma unroll
    for (int cbi = 0; cbi < 2; ++cbi) {
      const int col = col0 + (2 * wave + cbi) * 32 + l32;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int c = nbr * 32 + 8 * (v / 4) + 4 * lh + (v % 4);
        if (c < R) partY[((int64_t)rt * n_pad + col) * pR + c] = yacc[nbr][cbi][v];
      }
    }
}

// Two waves per SIMD (two work-groups per CU, which the LDS allows): the
// one-block form would otherwise take 258 registers and run one wave per SIMD.
template <int NB>
__global__ void __launch_bounds__(256, 2) k_skinny_bf16(const SkinnyDesc d) {
  skinny_body<NB>(static_cast<const uint16_t*>(d.src), d.ldp, d.n_pad, d.tile_rows, d.Uj, d.Vj, d.W, d.R, d.partX, d.partY, d.pR, blockIdx.x,
                  blockIdx.y);
}

// Index of the descriptor whose block range holds block b (sorted by
// block_begin, the first at 0).
__device__ __forceinline__ int find_skinny(const SkinnyDesc* __restrict__ ds, int nd, int b) {
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ds[mid].block_begin <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int NB>
__global__ void __launch_bounds__(256, 2) k_skinny_bf16_multi(const SkinnyDesc* __restrict__ ds, int nd) {
  const SkinnyDesc d = load_desc(ds, find_skinny(ds, nd, (int)blockIdx.x));
  const int local = (int)blockIdx.x - d.block_begin;
  skinny_body<NB>(static_cast<const uint16_t*>(d.src), d.ldp, d.n_pad, d.tile_rows, d.Uj, d.Vj, d.W, d.R, d.partX, d.partY, d.pR,
                  local % d.nct, local / d.nct);
}


// Update fused into the float skinny pass (R = 16 or 32 factor columns, one
// launch): blocks of 512 threads, waves 0-3 form X and Y on the matrix cores
// as the read-only pass does and waves 4-7 apply P += U_j V_j^T to the same
// chunk on the vector units: update wave wu takes rows wu + 4 i of the chunk
// and lane g the columns 4 g .. 4 g + 3; the old values come from the chunk
// in LDS, U_j rows of the chunk from sUr, V_j rows of the tile's columns
// from sVc (sVc[c][k] = V_j[col0 + k][c]); the delta is summed over c in
// order from zero and added once; the new rows go straight to HBM.  The
// matrix-core and vector work of a chunk share the SIMDs.
template <int CR, int SW, int UW>
__device__ __forceinline__ void chunk_update(float* __restrict__ P, const int64_t ldp, const int col0, const int cr0,
                                             const int R, const float (*sP)[SW], const float (*sUr)[UW],
                                             const float (*sVc)[SW], const int wu, const int lane) {
  float d[CR / 4][4];
#pragma unroll
  for (int i = 0; i < CR / 4; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) d[i][q] = 0.f;
  for (int c0 = 0; c0 < R; c0 += 4) {
    f32x4 v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = *reinterpret_cast<const f32x4*>(&sVc[c0 + e][4 * lane]);
#pragma unroll
    for (int i = 0; i < CR / 4; ++i) {
      const f32x4 u = *reinterpret_cast<const f32x4*>(&sUr[wu + 4 * i][c0]);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int q = 0; q < 4; ++q) d[i][q] = fma(u[e], v[e][q], d[i][q]);
    }
  }
#pragma unroll
  for (int i = 0; i < CR / 4; ++i) {
    f32x4 p = *reinterpret_cast<const f32x4*>(&sP[wu + 4 * i][4 * lane]);
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q] += d[i][q];
    __builtin_nontemporal_store(p, reinterpret_cast<f32x4*>(P + (int64_t)(cr0 + wu + 4 * i) * ldp + col0 + 4 * lane));
  }
}

// Float skinny pass.  Tile: about tile_rows x 256 columns of P, chunks of 32
// rows through LDS (the next chunk of P and V_j held in registers meanwhile);
// factor columns padded with zeros to 32 NB (NB <= 2).  The ns row slices of
// a column tile interleave by chunks (slice rt takes chunks rt, rt + ns, ...),
// so the grid streams one band of rows at a time.
//   X: the chunk's 32 x 32 NB outputs with K = 256 split over the waves
//      (wave w: columns [64 w, 64 w + 64)); the four partial sums meet in
//      LDS (over the chunk buffer, no longer read) and are added in wave
//      order; one partial per (row, column tile).
//   Y: as the bfloat16 kernel, wave w owns tile columns [64 w, 64 w + 64).
// A group of four f32 steps covers 8 summation indices: lanes 0-31 supply
// index g + e and lanes 32-63 index g + 4 + e in step e, for both operands.
// `want` selects the products formed (bit 0: X, bit 1: Y; uniform).
template <int NB, bool UPD = false>
__device__ __forceinline__ void skinny_f32_body(const float* __restrict__ P, const int64_t ldp, const int n_pad,
                                                const int tile_rows, const float* __restrict__ Uj,
                                                const float* __restrict__ Vj, const int W, const int R,
                                                float* __restrict__ partX, float* __restrict__ partY,
                                                const int pR, const int want, const int ct, const int rt) {
  const bool wx = (want & kWantX) != 0, wy = (want & kWantY) != 0;
  constexpr int RP = 32 * NB;
  constexpr int CR = 32;           // rows per chunk
  constexpr int FP = 4;            // LDS row padding (floats)
  constexpr int NT = UPD ? 512 : 256;
  static_assert(NB <= 2, "the X exchange buffer must fit in the chunk buffer");
  static_assert(!UPD || NB == 1, "the fused update takes all factor columns in one launch");
  __shared__ __align__(16) float sP[CR][TCB + FP];
  __shared__ __align__(16) float sUt[RP][TCB + FP];
  __shared__ __align__(16) float sVt[RP][CR + FP];
  __shared__ __align__(16) float sVc[UPD ? RP : 1][TCB + FP];
  __shared__ __align__(16) float sUr[UPD ? CR : 1][RP + FP];
  float* xbuf = &sP[0][0];         // [4 waves][NB][16 values][64 lanes]

  const int tid = threadIdx.x;
  const bool mwave = !UPD || tid < 256;   // matrix-core waves (all of them without the update)
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col0 = ct * TCB;
  // interleaved chunks: slice rt of ns takes chunks rt, rt + ns, ...
  const int ns = (n_pad + tile_rows - 1) / tile_rows;
  const int CS = ns * 32;
  const int row0 = rt * 32;
  const int rend = n_pad;
  const int l32 = lane % 32, lh = lane / 32;
  // chunk staging: thread -> rows tid / 64 + 4 i, f32x4 column group tid % 64
  const int srow = tid / 64, sgrp = tid % 64;

  constexpr int VPT = RP * CR / 256;
  f32x4 pre[CR / 4];
  float pv[VPT];
  auto fetch = [&](const int r0) {
    static_for<0, CR / 4>([&](auto i) {
      pre[i] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(P + (int64_t)(r0 + srow + 4 * i) * ldp + col0 +
                                                                     sgrp * 4));
    });
    static_for<0, VPT>([&](auto i) {
      const int idx = tid + 256 * i;
      const int rr = idx / RP, c = idx % RP;
      pv[i] = fac_clamped(Vj + (int64_t)(r0 + rr) * W, c, R);
    });
  };
  // update waves: the chunk's U_j rows (thread t = tid - 256 holds entries t + 256 i)
  float pu[VPT];
  auto fetch_u = [&](const int r0) {
    static_for<0, VPT>([&](auto i) {
      const int idx = tid - 256 + 256 * i;
      const int rr = idx / RP, c = idx % RP;
      pu[i] = fac_clamped(Uj + (int64_t)(r0 + rr) * W, c, R);
    });
  };
  if (mwave) fetch(row0);
  else if constexpr (UPD) fetch_u(row0);

  if (wx)
    batched_stage<RP * TCB / NT, NT, float>(
        tid, RP * TCB, [&](int idx) { const int c = idx % RP; return fac_or_zero(Uj + (int64_t)(col0 + idx / RP) * W, c, R); },
        [&](int idx, float v) { sUt[idx % RP][idx / RP] = v; });
  if constexpr (UPD)
    batched_stage<RP * TCB / NT, NT, float>(
        tid, RP * TCB, [&](int idx) { const int c = idx % RP; return fac_or_zero(Vj + (int64_t)(col0 + idx / RP) * W, c, R); },
        [&](int idx, float v) { sVc[idx % RP][idx / RP] = v; });

  v16f yacc[NB][2];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) yacc[a][b][v] = 0.f;

  for (int cr0 = row0; cr0 < rend; cr0 += CS) {
    __syncthreads();   // the previous chunk's exchange buffer has been read
    if (mwave) {
      static_for<0, CR / 4>([&](auto i) { *reinterpret_cast<f32x4*>(&sP[srow + 4 * i][sgrp * 4]) = pre[i]; });
      static_for<0, VPT>([&](auto i) {
        const int idx = tid + 256 * i;
        sVt[idx % RP][idx / RP] = idx % RP < R ? pv[i] : 0.f;
      });
    } else if constexpr (UPD) {
      static_for<0, VPT>([&](auto i) {
        const int idx = tid - 256 + 256 * i;
        sUr[idx / RP][idx % RP] = idx % RP < R ? pu[i] : 0.f;
      });
    }
    __syncthreads();
    if constexpr (UPD) {
      if (!mwave) {
        if (cr0 + CS < rend) fetch_u(cr0 + CS);
        chunk_update<CR, TCB + FP, RP + FP>(const_cast<float*>(P), ldp, col0, cr0, R, sP, sUr, sVc, wave - 4, lane);
        continue;
      }
    }
    if (cr0 + CS < rend) fetch(cr0 + CS);

    if constexpr (NB == 1) {
      // one 32-column factor block: wave w forms the 16 x 16 X tile of rows
      // 16 (w % 2) .. +15 and factor columns 16 (w / 2) .. +15 over the whole
      // tile width on v_mfma_f32_16x16x4f32 (lane l: row / column l % 16,
      // summation index g + 4 (l / 16) + e), so no partial sums cross waves
      if (wx) {
        typedef float v4f __attribute__((ext_vector_type(4)));
        const int l16 = lane % 16, lq = lane / 16;
        const int mb = wave % 2, nbx = wave / 2;
        v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
        for (int g = 0; g < TCB; g += 32) {
          const f32x4 a0 = *reinterpret_cast<const f32x4*>(&sP[mb * 16 + l16][g + 4 * lq]);
          const f32x4 b0 = *reinterpret_cast<const f32x4*>(&sUt[nbx * 16 + l16][g + 4 * lq]);
          const f32x4 a1 = *reinterpret_cast<const f32x4*>(&sP[mb * 16 + l16][g + 16 + 4 * lq]);
          const f32x4 b1 = *reinterpret_cast<const f32x4*>(&sUt[nbx * 16 + l16][g + 16 + 4 * lq]);
          acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.x, b0.x, acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.x, b1.x, acc1, 0, 0, 0);
          acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.y, b0.y, acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.y, b1.y, acc1, 0, 0, 0);
          acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.z, b0.z, acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.z, b1.z, acc1, 0, 0, 0);
          acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.w, b0.w, acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.w, b1.w, acc1, 0, 0, 0);
        }
        const int c = nbx * 16 + l16;
        if (c < R) {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            partX[((int64_t)ct * n_pad + cr0 + mb * 16 + 4 * lq + v) * pR + c] = acc0[v] + acc1[v];
        }
      }
    }
    // X partial over this wave's 64 columns (two factor blocks)
    v16f xacc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int v = 0; v < 16; ++v) xacc[nb][v] = 0.f;
#pragma unroll
    for (int g = 0; g < (wx && NB > 1 ? 64 : 0); g += 8) {
      const int k0 = wave * 64 + g + 4 * lh;
      const f32x4 a = *reinterpret_cast<const f32x4*>(&sP[l32][k0]);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const f32x4 b = *reinterpret_cast<const f32x4*>(&sUt[nb * 32 + l32][k0]);
        xacc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, xacc[nb], 0, 0, 0);
        xacc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, xacc[nb], 0, 0, 0);
        xacc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b.z, xacc[nb], 0, 0, 0);
        xacc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b.w, xacc[nb], 0, 0, 0);
      }
    }

    // Y^T += V_chunk^T P_chunk
#pragma unroll
    for (int g = 0; g < (wy ? CR : 0); g += 8) {
      const int r0 = g + 4 * lh;
#pragma unroll
      for (int cbi = 0; cbi < 2; ++cbi) {
        const int colc = (2 * wave + cbi) * 32 + l32;
        const float b0 = sP[r0][colc], b1 = sP[r0 + 1][colc], b2 = sP[r0 + 2][colc], b3 = sP[r0 + 3][colc];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          const f32x4 a = *reinterpret_cast<const f32x4*>(&sVt[nb * 32 + l32][r0]);
          yacc[nb][cbi] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b0, yacc[nb][cbi], 0, 0, 0);
          yacc[nb][cbi] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b1, yacc[nb][cbi], 0, 0, 0);
          yacc[nb][cbi] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b2, yacc[nb][cbi], 0, 0, 0);
          yacc[nb][cbi] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b3, yacc[nb][cbi], 0, 0, 0);
        }
      }
    }

    if (!wx || NB == 1) continue;
    // exchange the X partials (sP is no longer read in this chunk)
    __syncthreads();
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int v = 0; v < 16; ++v) xbuf[((wave * NB + nb) * 16 + v) * 64 + lane] = xacc[nb][v];
    __syncthreads();
    // thread -> (v, lane) slots of the 32 x 32 NB outputs
#pragma unroll
    for (int i = 0; i < NB * 4; ++i) {
      const int slot = tid + 256 * i;          // [nb][v][lane]
      const int ln = slot % 64, v = (slot / 64) % 16, nb = slot / 1024;
      float x = 0.f;
#pragma unroll
      for (int w = 0; w < 4; ++w) x += xbuf[((w * NB + nb) * 16 + v) * 64 + ln];
      const int c = nb * 32 + ln % 32;
      const int rr = 8 * (v / 4) + 4 * (ln / 32) + (v % 4);
      if (c < R) partX[((int64_t)ct * n_pad + cr0 + rr) * pR + c] = x;
    }
  }

  if (!wy || !mwave) return;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int cbi = 0; cbi < 2; ++cbi) {
      const int col = col0 + (2 * wave + cbi) * 32 + l32;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int c = nb * 32 + 8 * (v / 4) + 4 * lh + (v % 4);
        if (c < R) partY[((int64_t)rt * n_pad + col) * pR + c] = yacc[nb][cbi][v];
      }
    }
}

// Float skinny pass for at most 16 factor columns on v_mfma_f32_16x16x4f32:
// half the matrix-core work of the 32-wide pass at these ranks.  Tiling,
// chunk staging, the X exchange and the partial layouts as skinny_f32_body.
// 16x16x4 layouts: A (16 x 4): lane l holds A[l % 16][l / 16]; B (4 x 16):
// lane l holds B[l / 16][l % 16]; C: element v of lane l is
// C[4 (l / 16) + v][l % 16].  A group of four steps covers 16 summation
// indices: lane l supplies index g + 4 (l / 16) + e in step e, for both
// operands.
template <bool UPD = false>
__device__ __forceinline__ void skinny16_f32_body(const float* __restrict__ P, const int64_t ldp, const int n_pad,
                                                  const int tile_rows, const float* __restrict__ Uj,
                                                  const float* __restrict__ Vj, const int W, const int R,
                                                  float* __restrict__ partX, float* __restrict__ partY,
                                                  const int pR, const int want, const int ct, const int rt) {
  typedef float v4f __attribute__((ext_vector_type(4)));
  const bool wx = (want & kWantX) != 0, wy = (want & kWantY) != 0;
  constexpr int RP = 16;
  constexpr int CR = 32;           // rows per chunk
  constexpr int FP = 4;            // LDS row padding (floats)
  constexpr int NT = UPD ? 512 : 256;
  __shared__ __align__(16) float sP[CR][TCB + FP];
  __shared__ __align__(16) float sUt[RP][TCB + FP];
  __shared__ __align__(16) float sVt[RP][CR + FP];
  __shared__ __align__(16) float sVc[UPD ? RP : 1][TCB + FP];
  __shared__ __align__(16) float sUr[UPD ? CR : 1][RP + FP];
  float* xbuf = &sP[0][0];         // [4 waves][2 row blocks][4 values][64 lanes]

  const int tid = threadIdx.x;
  const bool mwave = !UPD || tid < 256;   // matrix-core waves (all of them without the update)
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col0 = ct * TCB;
  // interleaved chunks: slice rt of ns takes chunks rt, rt + ns, ...
  const int ns = (n_pad + tile_rows - 1) / tile_rows;
  const int CS = ns * 32;
  const int row0 = rt * 32;
  const int rend = n_pad;
  const int l16 = lane % 16, lq = lane / 16;
  const int srow = tid / 64, sgrp = tid % 64;

  constexpr int VPT = RP * CR / 256;
  f32x4 pre[CR / 4];
  float pv[VPT];
  auto fetch = [&](const int r0) {
    static_for<0, CR / 4>([&](auto i) {
      pre[i] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(P + (int64_t)(r0 + srow + 4 * i) * ldp + col0 +
                                                                     sgrp * 4));
    });
    static_for<0, VPT>([&](auto i) {
      const int idx = tid + 256 * i;
      const int rr = idx / RP, c = idx % RP;
      pv[i] = fac_clamped(Vj + (int64_t)(r0 + rr) * W, c, R);
    });
  };
  // update waves: the chunk's U_j rows (thread t = tid - 256 holds entries t + 256 i)
  float pu[VPT];
  auto fetch_u = [&](const int r0) {
    static_for<0, VPT>([&](auto i) {
      const int idx = tid - 256 + 256 * i;
      const int rr = idx / RP, c = idx % RP;
      pu[i] = fac_clamped(Uj + (int64_t)(r0 + rr) * W, c, R);
    });
  };
  if (mwave) fetch(row0);
  else if constexpr (UPD) fetch_u(row0);

  if (wx)
    batched_stage<RP * TCB / NT, NT, float>(
        tid, RP * TCB, [&](int idx) { const int c = idx % RP; return fac_or_zero(Uj + (int64_t)(col0 + idx / RP) * W, c, R); },
        [&](int idx, float v) { sUt[idx % RP][idx / RP] = v; });
  if constexpr (UPD)
    batched_stage<RP * TCB / NT, NT, float>(
        tid, RP * TCB, [&](int idx) { const int c = idx % RP; return fac_or_zero(Vj + (int64_t)(col0 + idx / RP) * W, c, R); },
        [&](int idx, float v) { sVc[idx % RP][idx / RP] = v; });

  v4f yacc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) yacc[cb] = v4f{0.f, 0.f, 0.f, 0.f};

  for (int cr0 = row0; cr0 < rend; cr0 += CS) {
    __syncthreads();   // the previous chunk's exchange buffer has been read
    if (mwave) {
      static_for<0, CR / 4>([&](auto i) { *reinterpret_cast<f32x4*>(&sP[srow + 4 * i][sgrp * 4]) = pre[i]; });
      static_for<0, VPT>([&](auto i) {
        const int idx = tid + 256 * i;
        sVt[idx % RP][idx / RP] = idx % RP < R ? pv[i] : 0.f;
      });
    } else if constexpr (UPD) {
      static_for<0, VPT>([&](auto i) {
        const int idx = tid - 256 + 256 * i;
        sUr[idx / RP][idx % RP] = idx % RP < R ? pu[i] : 0.f;
      });
    }
    __syncthreads();
    if constexpr (UPD) {
      if (!mwave) {
        if (cr0 + CS < rend) fetch_u(cr0 + CS);
        chunk_update<CR, TCB + FP, RP + FP>(const_cast<float*>(P), ldp, col0, cr0, R, sP, sUr, sVc, wave - 4, lane);
        if (wx) {              // the X exchange below overwrites the chunk: take part in its barriers
          __syncthreads();
          __syncthreads();
        }
        continue;
      }
    }
    if (cr0 + CS < rend) fetch(cr0 + CS);

    // X partial over this wave's 64 columns, two 16-row blocks
    v4f xacc[2] = {v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int g = 0; g < (wx ? 64 : 0); g += 16) {
      const int k0 = wave * 64 + g + 4 * lq;
      const f32x4 b = *reinterpret_cast<const f32x4*>(&sUt[l16][k0]);
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
        const f32x4 a = *reinterpret_cast<const f32x4*>(&sP[mb * 16 + l16][k0]);
        xacc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, xacc[mb], 0, 0, 0);
        xacc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, xacc[mb], 0, 0, 0);
        xacc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, xacc[mb], 0, 0, 0);
        xacc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, xacc[mb], 0, 0, 0);
      }
    }

    // Y^T += V_chunk^T P_chunk for this wave's four 16-column blocks
#pragma unroll
    for (int g = 0; g < (wy ? CR : 0); g += 16) {
      const int r0 = g + 4 * lq;
      const f32x4 a = *reinterpret_cast<const f32x4*>(&sVt[l16][r0]);
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int colc = wave * 64 + cb * 16 + l16;
        yacc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, sP[r0][colc], yacc[cb], 0, 0, 0);
        yacc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, sP[r0 + 1][colc], yacc[cb], 0, 0, 0);
        yacc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, sP[r0 + 2][colc], yacc[cb], 0, 0, 0);
        yacc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, sP[r0 + 3][colc], yacc[cb], 0, 0, 0);
      }
    }

    if (!wx) continue;
    // exchange the X partials (sP is no longer read in this chunk)
    __syncthreads();
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int v = 0; v < 4; ++v) xbuf[((wave * 2 + mb) * 4 + v) * 64 + lane] = xacc[mb][v];
    __syncthreads();
    // thread -> (row block, value, lane) slots of the 32 x 16 outputs
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int slot = tid + 256 * i;          // [mb][v][lane]
      const int ln = slot % 64, v = (slot / 64) % 4, mb = slot / 256;
      float x = 0.f;
#pragma unroll
      for (int w = 0; w < 4; ++w) x += xbuf[((w * 2 + mb) * 4 + v) * 64 + ln];
      const int c = ln % 16;
      const int rr = mb * 16 + 4 * (ln / 16) + v;
      if (c < R) partX[((int64_t)ct * n_pad + cr0 + rr) * pR + c] = x;
    }
  }

  if (!wy || !mwave) return;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int col = col0 + wave * 64 + cb * 16 + l16;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = 4 * lq + v;
      if (c < R) partY[((int64_t)rt * n_pad + col) * pR + c] = yacc[cb][v];
    }
  }
}

template <bool UPD>
__global__ void __launch_bounds__(UPD ? 512 : 256) k_skinny16_f32(const SkinnyDesc d) {
  skinny16_f32_body<UPD>(static_cast<const float*>(d.src), d.ldp, d.n_pad, d.tile_rows, d.Uj, d.Vj, d.W, d.R,
                         d.partX, d.partY, d.pR, d.want, blockIdx.x, blockIdx.y);
}

template <bool UPD>
__global__ void __launch_bounds__(UPD ? 512 : 256) k_skinny16_f32_multi(const SkinnyDesc* __restrict__ ds, int nd) {
  const SkinnyDesc d = load_desc(ds, find_skinny(ds, nd, (int)blockIdx.x));
  const int local = (int)blockIdx.x - d.block_begin;
  skinny16_f32_body<UPD>(static_cast<const float*>(d.src), d.ldp, d.n_pad, d.tile_rows, d.Uj, d.Vj, d.W, d.R,
                         d.partX, d.partY, d.pR, d.want, local % d.nct, local / d.nct);
}

template <int NB, bool UPD>
__global__ void __launch_bounds__(UPD ? 512 : 256) k_skinny_f32(const SkinnyDesc d) {
  skinny_f32_body<NB, UPD>(static_cast<const float*>(d.src), d.ldp, d.n_pad, d.tile_rows, d.Uj, d.Vj, d.W, d.R,
                           d.partX, d.partY, d.pR, d.want, blockIdx.x, blockIdx.y);
}

template <int NB, bool UPD>
__global__ void __launch_bounds__(UPD ? 512 : 256) k_skinny_f32_multi(const SkinnyDesc* __restrict__ ds, int nd) {
  const SkinnyDesc d = load_desc(ds, find_skinny(ds, nd, (int)blockIdx.x));
  const int local = (int)blockIdx.x - d.block_begin;
  skinny_f32_body<NB, UPD>(static_cast<const float*>(d.src), d.ldp, d.n_pad, d.tile_rows, d.Uj, d.Vj, d.W, d.R,
                           d.partX, d.partY, d.pR, d.want, local % d.nct, local / d.nct);
}

// X-only float pass on the matrix cores: partial X = P U for R <= 16 NB
// factor columns (zero-padded), P streamed from HBM straight into the MFMA
// operand registers: no LDS staging of P, no exchange between waves.
// Block: kXWaves waves over kXRows rows x 256 columns of P; wave w takes
// the 16-row strips w, w + kXWaves, ..., each read in two halves of 128
// columns, the next half requested before the current one is multiplied.
// v_mfma_f32_16x16x4f32: A (16 x 4): lane l holds A[l % 16][l / 16];
// B (4 x 16): lane l holds B[l / 16][l % 16]; C: element v of lane l is
// C[4 (l / 16) + v][l % 16].  In a 32-column group, lane l reads 4 floats
// of strip row l % 16 at column 4 (l / 16) and 4 at column 16 + 4 (l / 16)
// (each load a contiguous 64-byte segment per row); step e of the group's
// 8 products takes the e-th of these floats as its summation index, and the
// B operand the matching U row.
constexpr int kXWaves = 8;
constexpr int kXRows = 512;
constexpr int XUS = 4;   // LDS row padding of the U tile (floats): rows 4 apart in distinct banks

template <int NB>
__global__ void __launch_bounds__(64 * kXWaves) k_xprod_f32(const SkinnyDesc d) {
  constexpr int RP = 16 * NB;
  __shared__ float sU[TCB][RP + XUS];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane % 16, lq = lane / 16;
  const int ct = blockIdx.x;
  const int col0 = ct * TCB;
  const int row0 = blockIdx.y * kXRows;
  const int nstrips = (min(row0 + kXRows, d.n_pad) - row0) / 16;
  const float* __restrict__ P = static_cast<const float*>(d.src);

  f32x4 bufA[4][2], bufB[4][2];
  auto load_half = [&](f32x4 (&b)[4][2], const int r, const int h) {
    const float* src = P + (int64_t)(r + l16) * d.ldp + col0 + 128 * h + 4 * lq;
    static_for<0, 4>([&](auto g) {
      b[g][0] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(src + 32 * g));
      b[g][1] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(src + 32 * g + 16));
    });
  };
  batched_stage<TCB * RP / (64 * kXWaves), 64 * kXWaves, float>(
      tid, TCB * RP,
      [&](int idx) { const int c = idx % RP; return c < d.R ? d.Uj[(int64_t)(col0 + idx / RP) * d.W + c] : 0.f; },
      [&](int idx, float v) { sU[idx / RP][idx % RP] = v; });
  __syncthreads();

  typedef float v4f __attribute__((ext_vector_type(4)));
  v4f acc[NB];
  auto multiply = [&](f32x4 (&b)[4][2], const int h) {
    static_for<0, 4>([&](auto g) {
      static_for<0, 8>([&](auto e) {
        const float a = e < 4 ? b[g][0][e % 4] : b[g][1][e % 4];
        const int k = 128 * h + 32 * g + 4 * lq + (e < 4 ? e : 12 + e);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, sU[k][nb * 16 + l16], acc[nb], 0, 0, 0);
      });
    });
  };

  if (wave < nstrips) load_half(bufA, row0 + 16 * wave, 0);
  for (int st = wave; st < nstrips; st += kXWaves) {
    const int r = row0 + 16 * st;
    // U operands are re-read from LDS in every strip: held in registers across
    // strips (as the compiler would otherwise do) they cost the occupancy
    asm volatile("" ::: "memory");
    load_half(bufB, r, 1);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) acc[nb] = v4f{0.f, 0.f, 0.f, 0.f};
    multiply(bufA, 0);
    if (st + kXWaves < nstrips) load_half(bufA, r + 16 * kXWaves, 0);
    multiply(bufB, 1);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int c = nb * 16 + l16;
      if (c < d.R) {
#pragma unroll
        for (int v = 0; v < 4; ++v) d.partX[((int64_t)ct * d.n_pad + r + 4 * lq + v) * d.pR + c] = acc[nb][v];
      }
    }
  }
}

__global__ void __launch_bounds__(256)
k_to_bf16(const float* __restrict__ P, uint16_t* __restrict__ S, int64_t count, const int* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (i >= count) return;
  const float4 p = *reinterpret_cast<const float4*>(P + i);
  ushort4 sh;
  sh.x = bf16_rne(p.x); sh.y = bf16_rne(p.y); sh.z = bf16_rne(p.z); sh.w = bf16_rne(p.w);
  *reinterpret_cast<ushort4*>(S + i) = sh;
}

}  // namespace

hipError_t launch_skinny_bf16(int R, const uint16_t* S, int64_t ldp, int64_t n_pad, int tile_rows,
                              const float* slabU, const float* slabV, int W, float* partX, float* partY,
                              hipStream_t s) {
  if (R < 1 || R > kMaxLevelRank || (R > 64 && R % 64 != 0) || n_pad % TCB != 0 || tile_rows % CRB != 0)
    return hipErrorInvalidValue;
  const int nct = (int)(n_pad / TCB);
  const dim3 grid((unsigned)nct, (unsigned)((n_pad + tile_rows - 1) / tile_rows));
  const float* Vj = slabV + (W - R);
  // at most 64 factor columns per launch: two launches of the two-block
  // kernel for R = 128 read the shadow twice but run at twice the occupancy
  // of one four-block launch (whose LDS allows one block per CU)
  const int per = R <= 64 ? R : 64;
  for (int c0 = 0; c0 < R; c0 += per) {
    const SkinnyDesc d{S, ldp, (int)n_pad, tile_rows, slabU + c0, Vj + c0, W, per, partX + c0, partY + c0, R, nct, 0};
    if (skinny_blocks_for(per) == 1)
      hipLaunchKernelGGL((k_skinny_bf16<1>), grid, dim3(256), 0, s, d);
    else
      hipLaunchKernelGGL((k_skinny_bf16<2>), grid, dim3(256), 0, s, d);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_skinny_bf16_multi(int nb, const SkinnyDesc* ds, int nd, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  switch (nb) {
    case 1: hipLaunchKernelGGL((k_skinny_bf16_multi<1>), dim3((unsigned)blocks), dim3(256), 0, s, ds, nd); break;
    case 2: hipLaunchKernelGGL((k_skinny_bf16_multi<2>), dim3((unsigned)blocks), dim3(256), 0, s, ds, nd); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_skinny_f32(int R, const float* P, int64_t ldp, int64_t n_pad, int tile_rows,
                             const float* slabU, const float* slabV, int W, float* partX, float* partY,
                             hipStream_t s, int want, bool update) {
  if (R < 1 || R > kMaxLevelRank || (R > 64 && R % 64 != 0) || n_pad % TCB != 0 || tile_rows % 32 != 0)
    return hipErrorInvalidValue;
  if (update) {
    // one launch over all R columns with the update fused (X and Y both)
    if (!skinny_update_kernel(R) || want != (kWantX | kWantY)) return hipErrorInvalidValue;
    const int nct = (int)(n_pad / TCB);
    const dim3 grid((unsigned)nct, (unsigned)((n_pad + tile_rows - 1) / tile_rows));
    const SkinnyDesc d{P, ldp, (int)n_pad, tile_rows, slabU, slabV + (W - R), W, R, partX, partY, R, nct, 0, want};
    if (R <= 16)
      hipLaunchKernelGGL(k_skinny16_f32<true>, grid, dim3(512), 0, s, d);
    else
      hipLaunchKernelGGL((k_skinny_f32<1, true>), grid, dim3(512), 0, s, d);
    return hipGetLastError();
  }
  if (want == kWantX) {
    // X only: the direct-operand pass (row tiling of its own; the X partials
    // do not depend on it)
    const int nct = (int)(n_pad / TCB);
    const dim3 grid((unsigned)nct, (unsigned)((n_pad + kXRows - 1) / kXRows));
    const int per = R <= 64 ? R : 64;
    for (int c0 = 0; c0 < R; c0 += per) {
      const SkinnyDesc d{P, ldp, (int)n_pad, kXRows, slabU + c0, nullptr, W, per, partX + c0, nullptr, R, nct, 0,
                         kWantX};
      if (per <= 16)
        hipLaunchKernelGGL((k_xprod_f32<1>), grid, dim3(64 * kXWaves), 0, s, d);
      else if (per <= 32)
        hipLaunchKernelGGL((k_xprod_f32<2>), grid, dim3(64 * kXWaves), 0, s, d);
      else
        hipLaunchKernelGGL((k_xprod_f32<4>), grid, dim3(64 * kXWaves), 0, s, d);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int nct = (int)(n_pad / TCB);
  const dim3 grid((unsigned)nct, (unsigned)((n_pad + tile_rows - 1) / tile_rows));
  const float* Vj = slabV + (W - R);
  // at most 32 factor columns per launch: the one-block kernel (two blocks
  // per CU, no X exchange) twice beats the two-block kernel (one per CU)
  const int per = R <= 32 ? R : 32;
  for (int c0 = 0; c0 < R; c0 += per) {
    const SkinnyDesc d{P, ldp, (int)n_pad, tile_rows, slabU + c0, Vj + c0, W, per, partX + c0, partY + c0, R, nct, 0,
                       want};
    if (skinny_f32_blocks(per) == 0)
      hipLaunchKernelGGL(k_skinny16_f32<false>, grid, dim3(256), 0, s, d);
    else
      hipLaunchKernelGGL((k_skinny_f32<1, false>), grid, dim3(256), 0, s, d);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_skinny_f32_multi(int nb, const SkinnyDesc* ds, int nd, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  switch (nb) {
    case 0: hipLaunchKernelGGL(k_skinny16_f32_multi<false>, dim3((unsigned)blocks), dim3(256), 0, s, ds, nd); break;
    case 1: hipLaunchKernelGGL((k_skinny_f32_multi<1, false>), dim3((unsigned)blocks), dim3(256), 0, s, ds, nd); break;
    case 2: hipLaunchKernelGGL(k_skinny16_f32_multi<true>, dim3((unsigned)blocks), dim3(512), 0, s, ds, nd); break;
    case 3: hipLaunchKernelGGL((k_skinny_f32_multi<1, true>), dim3((unsigned)blocks), dim3(512), 0, s, ds, nd); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float* P, uint16_t* S, int64_t count, hipStream_t s, const int* gate) {
  if (count % 4 != 0) return hipErrorInvalidValue;
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((count / 4 + 255) / 256)), dim3(256), 0, s, P, S, count, gate);
  return hipGetLastError();
}

}  // namespace lv
