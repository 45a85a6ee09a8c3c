// BF16-shadow form of a level (storage FP32).  Every stored power P_j below
// the top keeps a bfloat16 copy S_j, rewritten by the update pass that adds
// U_j V_j^T to P_j.  The level's skinny products (App. A, with the OLD power)
// are formed from the shadow on the matrix cores:
//     X = S_j U_j,   Y^T = V_j^T S_j      (bf16 x bf16 -> fp32 accumulation)
// reading 2 bytes per element of the power instead of 4.  The partial X / Y
// layouts are those of the FP32 fused pass, so the FP32 tail assembles the
// next factors; the Gram V_j^T U_j is formed in FP64 by its own kernel.
//
// Lane layouts of v_mfma_f32_32x32x16_bf16 (64 lanes, l = lane):
//   A (32 x 16): lane l holds A[l % 32][8 (l / 32) + e], e = 0..7
//   B (16 x 32): lane l holds B[8 (l / 32) + e][l % 32]
//   C (32 x 32): element v of lane l is C[8 (v / 4) + 4 (l / 32) + v % 4][l % 32]
#include "lv_internal.h"

namespace lv {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int TCB = 256;   // tile columns
constexpr int CRB = 64;    // rows per LDS chunk
constexpr int SPAD = 8;    // LDS row padding (bf16 elements, keeps 16-byte alignment)

__device__ __forceinline__ bf16x8 lds8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(p));
}

// Tile: tile_rows x 256 columns of S, walked in chunks of 64 rows through
// LDS, the next chunk held in registers while the current one is used.
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
  const int row0 = rt * tile_rows;
  const int rend = min(row0 + tile_rows, n_pad);
  const int l32 = lane % 32, lh = lane / 32;
  // chunk staging: thread -> rows tid / 32 + 8 i, 16-byte column group tid % 32
  const int srow = tid / 32, sgrp = tid % 32;

  u16x8 pre[CRB / 8];
#pragma unroll
  for (int i = 0; i < CRB / 8; ++i)
    pre[i] = *reinterpret_cast<const u16x8*>(S + (int64_t)(row0 + srow + 8 * i) * ldp + col0 + sgrp * 8);

  // U_j rows of the tile's columns, transposed: sUt[c][k] = U_j[col0 + k][c]
  for (int idx = tid; idx < RP * TCB; idx += 256) {
    const int k = idx / RP, c = idx % RP;
    sUt[c][k] = c < R ? bf16_rne(Uj[(int64_t)(col0 + k) * W + c]) : (uint16_t)0;
  }

  v16f yacc[NB][2];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) yacc[a][b][v] = 0.f;

  for (int cr0 = row0; cr0 < rend; cr0 += CRB) {
    __syncthreads();   // the previous chunk is no longer read
#pragma unroll
    for (int i = 0; i < CRB / 8; ++i) *reinterpret_cast<u16x8*>(&sS[srow + 8 * i][sgrp * 8]) = pre[i];
    for (int idx = tid; idx < RP * CRB; idx += 256) {
      const int rr = idx / RP, c = idx % RP;
      sVt[c][rr] = c < R ? bf16_rne(Vj[(int64_t)(cr0 + rr) * W + c]) : (uint16_t)0;
    }
    __syncthreads();
    if (cr0 + CRB < rend) {
#pragma unroll
      for (int i = 0; i < CRB / 8; ++i)
        pre[i] = *reinterpret_cast<const u16x8*>(S + (int64_t)(cr0 + CRB + srow + 8 * i) * ldp + col0 + sgrp * 8);
    }

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

template <int NB>
__global__ void __launch_bounds__(256) k_skinny_bf16(const SkinnyDesc d) {
  skinny_body<NB>(d.S, d.ldp, d.n_pad, d.tile_rows, d.Uj, d.Vj, d.W, d.R, d.partX, d.partY, d.pR, blockIdx.x,
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
__global__ void __launch_bounds__(256) k_skinny_bf16_multi(const SkinnyDesc* __restrict__ ds, int nd) {
  const SkinnyDesc d = ds[find_skinny(ds, nd, (int)blockIdx.x)];
  const int local = (int)blockIdx.x - d.block_begin;
  skinny_body<NB>(d.S, d.ldp, d.n_pad, d.tile_rows, d.Uj, d.Vj, d.W, d.R, d.partX, d.partY, d.pR,
                  local % d.nct, local / d.nct);
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
  if (R < 1 || R > 128 || n_pad % TCB != 0 || tile_rows % CRB != 0) return hipErrorInvalidValue;
  const int nct = (int)(n_pad / TCB);
  const SkinnyDesc d{S, ldp, (int)n_pad, tile_rows, slabU, slabV + (W - R), W, R, partX, partY, R, nct, 0};
  const dim3 grid((unsigned)nct, (unsigned)((n_pad + tile_rows - 1) / tile_rows));
  switch (skinny_blocks_for(R)) {
    case 1: hipLaunchKernelGGL((k_skinny_bf16<1>), grid, dim3(256), 0, s, d); break;
    case 2: hipLaunchKernelGGL((k_skinny_bf16<2>), grid, dim3(256), 0, s, d); break;
    default: hipLaunchKernelGGL((k_skinny_bf16<4>), grid, dim3(256), 0, s, d); break;
  }
  return hipGetLastError();
}

hipError_t launch_skinny_bf16_multi(int nb, const SkinnyDesc* ds, int nd, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  switch (nb) {
    case 1: hipLaunchKernelGGL((k_skinny_bf16_multi<1>), dim3((unsigned)blocks), dim3(256), 0, s, ds, nd); break;
    case 2: hipLaunchKernelGGL((k_skinny_bf16_multi<2>), dim3((unsigned)blocks), dim3(256), 0, s, ds, nd); break;
    case 4: hipLaunchKernelGGL((k_skinny_bf16_multi<4>), dim3((unsigned)blocks), dim3(256), 0, s, ds, nd); break;
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
