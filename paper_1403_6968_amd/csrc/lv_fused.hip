// Fused level pass of the IncrExp update (LINVIEW, App. A exponential model).
//
// For one level j of the exponential model the update needs, with the OLD
// stored power P = A^(2^j) and the level factors U_j, V_j (n x R, R = 2^j r):
//     X = P U_j,   Y = P^T V_j,   G = V_j^T U_j,   P += U_j V_j^T
// and then U_{j+1} = [U_j, X + U_j G], V_{j+1} = [Y, V_j]  (Sec. 4.3, App. A).
//
// k_level_fused does the first four in ONE read and ONE write of P: a tile of
// P is streamed through registers once; Y and the rank-R update use the
// coalesced row-segment layout directly, and the old values go through LDS
// so that X can be formed with one row per lane (no cross-lane reductions).
// Each tile writes partial X / Y (and the column-tile-0 tiles partial Grams);
// k_level_tail reduces them in a fixed order (deterministic, no float
// atomics) and assembles the next level's factors.  k_level_update is the
// update-only pass of the top stored power.
//
// Layouts (all row-major):
//   P        n_pad x ldp, zero padding beyond n.
//   slab U   n_pad x W; U_j = columns [0, R).
//   slab V   n_pad x W; V_j = columns [W - R, W)  (callers pass the offset base).
//   partX    [nct][n_pad][R]   (nct = n_pad / TC column tiles)
//   partY    [nrt][n_pad][R]   (nrt row tiles)
//   partG    [nrt][R][R] double
#include "lv_device.h"

namespace lv {
namespace {

// ---------------------------------------------------------------- fused pass
//
// Block: 256 threads (4 waves).  Columns: TC = 64 lanes x 16 B.  Rows: the
// matrix is cut into blocks of RB rows, and the ns = ceil(n_pad / tile_rows)
// row slices of a column tile interleave: slice s owns the row blocks
// b = s, s + ns, s + 2 ns, ... (about tile_rows rows in all), and its wave w
// the i-th of them for i = w, w + 4, w + 8, ...  At any moment the grid thus
// streams one contiguous band of rows rather than ns bands a tile apart,
// which the HBM serves at a markedly higher rate.  Each wave processes its
// blocks end to end with no block-wide synchronisation:
//   Phase A  one 16-byte vector per lane per row: Y partial (yacc, the
//            lane's own columns, V_j rows broadcast through the scalar unit),
//            the old values to the wave's private LDS block, and
//            P + U_j V_j^T back to HBM; the next block's rows are then
//            requested at once so that they are in flight during Phase B.
//   Phase B  lane (rho, q) = (lane % RB, lane / RB) sums row rho of the block
//            over the q-th of NQ = 64 / RB column slices with the tile's
//            U_j rows read from LDS (staged once per tile); the NQ slice
//            sums are combined with xor-shuffles and one partial per
//            (row, tile column) is written.
// The four waves' Y accumulators are summed once at the end of the tile.
//
// UPD = false gives the read-only variant used for ranks above 16: the
// skinny products of 16 factor columns at a time (partials written with row
// stride pR at the chunk's column offset), the rank update and the Gram done
// by k_level_update and k_gram.
//
// Variants for views that keep the sums of powers or a general form as well
// (one pass over a stored matrix instead of two or three):
//   XE, XD   X is formed for XE + XD more columns: XE taken from Ux (same
//            stride W), XD from Ud (stride Wd), X = P [U_j, Q_j, D_j]; the
//            extra blocks' partials go to partX2 (row stride XE) and partX3
//            (row stride XD).  The powers' pass thus also yields P_j Q_j
//            (sums) and P_j D_j (the general form's delta or factor slab).
//   SP       the sums pass: no X; Y = S^T Vy with the old S and the rank
//            update S += Uj Vj^T (Uj = Q_j, Vj = W_j), no Gram.
template <typename T, int R, int RB, bool UPD, int XE = 0, bool SP = false, int XD = 0>
__device__ __forceinline__ void fused_body(T* __restrict__ P, const int64_t ldp, const int n_pad,
                                           const int tile_rows, const T* __restrict__ Uj,
                                           const T* __restrict__ Vj, const int W, T* __restrict__ partX,
                                           T* __restrict__ partY, double* __restrict__ partG, const int pR,
                                           const int ct, const int rt, const T* __restrict__ Ux = nullptr,
                                           T* __restrict__ partX2 = nullptr, const T* __restrict__ Vy = nullptr,
                                           const T* __restrict__ Ud = nullptr, const int Wd = 0,
                                           T* __restrict__ partX3 = nullptr) {
  constexpr int EPL = 16 / (int)sizeof(T);
  constexpr int TC = 64 * EPL;
  constexpr int NQ = 64 / RB;           // column slices in Phase B
  constexpr int QW = TC / NQ;           // columns per slice
  constexpr int LDSW = TC + EPL;        // padded LDS row (elements)
  constexpr int UPAD = 4;               // LDS padding between U slices (elements)
  constexpr int XR = R + XE + XD;       // columns of X
  static_assert(!SP || (UPD && XE == 0 && XD == 0), "the sums pass updates and forms no X");
  // Phase B on the matrix cores (float, 8-row blocks, X at most 16 columns):
  // there the vector units would carry the three products of the pass.
  constexpr bool MFX = sizeof(T) == 4 && RB == 8 && XR <= 16 && !SP;
  constexpr int UTW = TC + 4;           // row of the transposed U tile (MFX)

  __shared__ __align__(16) T tileP[4 * RB * LDSW];
  __shared__ __align__(16) T utile[SP ? 1 : MFX ? 16 * UTW : TC * XR + NQ * UPAD];
  // per wave: the current row block's factor entries (Y operand, then U_j),
  // row-major RB x R each, read back as wave-uniform broadcasts
  constexpr int FB = RB * R;
  __shared__ __align__(16) T facs[4][UPD ? 2 : 1][FB];
  // MFX: a zero row that supplies the A operand of the rows RB..15
  __shared__ __align__(16) float zrow[MFX ? TC : 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = wave_id();
  const int col0 = ct * TC;
  const int ns = (n_pad + tile_rows - 1) / tile_rows;   // row slices
  const int nb_all = n_pad / RB;
  const int nblocks = (nb_all - rt + ns - 1) / ns;      // row blocks of slice rt
  // first row of the slice's i-th row block
  auto blk_row = [&](int i) -> int64_t { return (int64_t)(rt + ns * i) * RB; };
  const int lc = col0 + lane * EPL;
  T* myP = tileP + wave * RB * LDSW;
  const T* __restrict__ Yop = SP ? Vy : Vj;

  // The block's factor rows (Y operand and, with the update, U_j): entry
  // e = t R + c of the RB x R block sits in lane e % 64 of fy[e / 64] (fu),
  // fetched with one gathered vector load per 64 entries together with the
  // block's rows of P; the wave writes them to its LDS block and reads them
  // back row by row as broadcasts (no scalar load, and so no scalar-cache
  // round trip, on the row loop, and no VALU work to broadcast).  PD blocks
  // beyond the current one are in flight while it is processed (slots
  // 1..PD); the first ones are requested before the tile's operands are
  // staged.
  constexpr int FN = (RB * R + 63) / 64;
  constexpr int PD = fused_prefetch(R);
  V16<T> pb[PD + 1][RB];
  T fyb[PD + 1][FN], fub[PD + 1][UPD ? FN : 1];
  auto load_block = [&](int slot, int64_t r0) {
#pragma unroll
    for (int t = 0; t < RB; ++t) pb[slot][t] = ld16_nt(P + (r0 + t) * ldp + lc);
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      const int e = lane + 64 * f;
      const int64_t o = (r0 + (e < RB * R ? e / R : 0)) * W + (e < RB * R ? e % R : 0);
      fyb[slot][f] = Yop[o];
      if constexpr (UPD) fub[slot][f] = Uj[o];
    }
  };
#pragma unroll
  for (int d = 0; d < (PD > 0 ? PD : 1); ++d)
    if (wave + 4 * d < nblocks) load_block(d, blk_row(wave + 4 * d));
  V16<T>* p = pb[0];
  T* fy = fyb[0];
  T* fu = fub[0];

  // X operand rows of the tile's columns, slice-padded: (col, c) -> col*XR + (col/QW)*UPAD + c;
  // for MFX transposed, (col, c) -> c*UTW + col, columns XR..15 zero.
  auto xop = [&](const int col, const int c) -> T {   // X operand (col, c), zero beyond XR
    const int64_t g = (int64_t)(col0 + col) * W;
    return c < R ? Uj[g + c]
         : c < R + XE ? Ux[g + c - R]
         : c < XR ? Ud[(int64_t)(col0 + col) * Wd + c - R - XE] : T(0);
  };
  if constexpr (MFX) {
    for (int idx = tid; idx < TC; idx += 256) zrow[idx] = 0.f;
    batched_stage<(TC * 16 + 255) / 256, 256, T>(
        tid, TC * 16, [&](int idx) { return xop(idx / 16, idx % 16); },
        [&](int idx, T v) { utile[(idx % 16) * UTW + idx / 16] = v; });
  } else if constexpr (!SP) {
    batched_stage<(TC * XR + 255) / 256, 256, T>(
        tid, TC * XR, [&](int idx) { return xop(idx / XR, idx % XR); },
        [&](int idx, T v) {
          const int col = idx / XR;
          utile[col * XR + (col / QW) * UPAD + idx % XR] = v;
        });
  }
  T vcol[EPL][UPD ? R : 1];
  if constexpr (UPD) {
#pragma unroll
    for (int q = 0; q < EPL; ++q)
#pragma unroll
      for (int c = 0; c < R; ++c) vcol[q][c] = Vj[(int64_t)(lc + q) * W + c];
  }

  T yacc[EPL][R];
#pragma unroll
  for (int q = 0; q < EPL; ++q)
#pragma unroll
    for (int c = 0; c < R; ++c) yacc[q][c] = T(0);

  __syncthreads();

  const int rho = lane % RB;
  const int qs = lane / RB;
  const T* urow0 = utile + qs * (QW * XR + UPAD);

  T* fac_y = facs[wave][0];
  T* fac_u = facs[wave][UPD ? 1 : 0];
  for (int b = wave; b < nblocks; b += 4) {
    const int64_t r0 = blk_row(b);
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      if (lane + 64 * f < FB) {
        fac_y[lane + 64 * f] = fy[f];
        if constexpr (UPD) fac_u[lane + 64 * f] = fu[f];
      }
    }
    if constexpr (PD > 0) {
      if (b + 4 * PD < nblocks) load_block(PD, blk_row(b + 4 * PD));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

#pragma unroll
    for (int t = 0; t < RB; ++t) {
      const int64_t i = r0 + t;
      T vi[R];
#pragma unroll
      for (int c = 0; c < R; ++c) vi[c] = fac_y[t * R + c];
#pragma unroll
      for (int q = 0; q < EPL; ++q)
#pragma unroll
        for (int c = 0; c < R; ++c) yacc[q][c] = fma(p[t].v[q], vi[c], yacc[q][c]);
      if constexpr (!SP) st16(myP + t * LDSW + lane * EPL, p[t]);
      if constexpr (UPD) {
        T ui[R];
#pragma unroll
        for (int c = 0; c < R; ++c) ui[c] = fac_u[t * R + c];
#pragma unroll
        for (int q = 0; q < EPL; ++q) {
          T d = ui[0] * vcol[q][0];
#pragma unroll
          for (int c = 1; c < R; ++c) d = fma(ui[c], vcol[q][c], d);
          p[t].v[q] += d;
        }
        st16_nt(P + i * ldp + lc, p[t]);
      }
    }
    // the next block moves into slot 0 (register moves; with PD = 0 it is
    // requested only now, while X of this block is formed)
    if constexpr (PD == 0) {
      if (b + 4 < nblocks) load_block(0, blk_row(b + 4));
    } else {
#pragma unroll
      for (int d = 0; d < PD; ++d) {
#pragma unroll
        for (int t = 0; t < RB; ++t) pb[d][t] = pb[d + 1][t];
#pragma unroll
        for (int f = 0; f < FN; ++f) {
          fyb[d][f] = fyb[d + 1][f];
          if constexpr (UPD) fub[d][f] = fub[d + 1][f];
        }
      }
    }
    if constexpr (SP) continue;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    if constexpr (MFX) {
      // X_block (16 x 16, rows RB..15 zero) = P_block U_tile on
      // v_mfma_f32_16x16x4f32: lane l supplies row l % 16 of the block and
      // U column l % 16, summation index 16 j + 4 (l / 16) + e in step e of
      // group j (two accumulators, even and odd groups, added at the end);
      // element v of lane l is X[4 (l / 16) + v][l % 16].
      typedef float v4f __attribute__((ext_vector_type(4)));
      const int l16 = lane % 16, lq = lane / 16;
      v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
      // lanes of rows RB..15 read the zero row
      const float* arow = (l16 < RB ? reinterpret_cast<const float*>(myP) + l16 * LDSW : zrow) + 4 * lq;
      const float* brow = reinterpret_cast<const float*>(utile) + l16 * UTW + 4 * lq;
#pragma unroll
      for (int j = 0; j < TC / 16; j += 2) {
        const V16<float> a0 = ld16(arow + 16 * j);
        const V16<float> b0 = ld16(brow + 16 * j);
        const V16<float> a1 = ld16(arow + 16 * j + 16);
        const V16<float> b1 = ld16(brow + 16 * j + 16);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.v[e], b0.v[e], acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1.v[e], b1.v[e], acc1, 0, 0, 0);
        }
      }
      if (lq < RB / 4) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = r0 + 4 * lq + v;
          const float xv = acc0[v] + acc1[v];
          if (l16 < R) partX[((int64_t)ct * n_pad + row) * pR + l16] = xv;
          if constexpr (XE > 0)
            if (l16 >= R && l16 < R + XE) partX2[((int64_t)ct * n_pad + row) * XE + l16 - R] = xv;
          if constexpr (XD > 0)
            if (l16 >= R + XE && l16 < XR) partX3[((int64_t)ct * n_pad + row) * XD + l16 - R - XE] = xv;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      continue;
    }

    T x[XR];
#pragma unroll
    for (int c = 0; c < XR; ++c) x[c] = T(0);
    const T* prow = myP + rho * LDSW + qs * QW;
#pragma unroll 4
    for (int l = 0; l < QW; l += EPL) {
      const V16<T> pv = ld16(prow + l);
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        const T* ur = urow0 + (l + e) * XR;
#pragma unroll
        for (int c = 0; c < XR; ++c) x[c] = fma(pv.v[e], ur[c], x[c]);
      }
    }
#pragma unroll
    for (int off = RB; off < 64; off <<= 1)
#pragma unroll
      for (int c = 0; c < XR; ++c) x[c] += __shfl_xor(x[c], off);
    if (qs == 0) {
#pragma unroll
      for (int c = 0; c < R; ++c) partX[((int64_t)ct * n_pad + r0 + rho) * pR + c] = x[c];
      if constexpr (XE > 0) {
#pragma unroll
        for (int c = 0; c < XE; ++c) partX2[((int64_t)ct * n_pad + r0 + rho) * XE + c] = x[R + c];
      }
      if constexpr (XD > 0) {
#pragma unroll
        for (int c = 0; c < XD; ++c) partX3[((int64_t)ct * n_pad + r0 + rho) * XD + c] = x[R + XE + c];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }

  // Y partial of this tile: sum the four waves' accumulators (in column
  // chunks of YC factor columns when the tile buffer cannot hold all R).
  constexpr int YCAP = (RB * LDSW) / TC;
  constexpr int YC = R < YCAP ? R : YCAP;
  static_assert(YC >= 1 && R % YC == 0, "Y reduction chunking");
  T* ybuf = tileP;
#pragma unroll
  for (int c0 = 0; c0 < R; c0 += YC) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < EPL; ++q)
#pragma unroll
      for (int c = 0; c < YC; ++c) ybuf[(wave * TC + lane * EPL + q) * YC + c] = yacc[q][c0 + c];
    __syncthreads();
    for (int idx = tid; idx < TC * YC; idx += 256) {
      const int cc = idx / YC, c = idx % YC;
      const T s = ((ybuf[(0 * TC + cc) * YC + c] + ybuf[(1 * TC + cc) * YC + c]) +
                   ybuf[(2 * TC + cc) * YC + c]) + ybuf[(3 * TC + cc) * YC + c];
      partY[((int64_t)rt * n_pad + col0 + cc) * pR + c0 + c] = s;
    }
  }

  // Partial Gram V_j^T U_j over this slice's rows (double accumulation).
  // The R^2 pairs are spread over the column tiles (pair p on column tile
  // p mod nct), so no block carries much more work than the others; for
  // the pairs of its tile, thread (pair, group) sums every G-th row of the
  // slice (counted in slice order) and the groups are then added in a fixed
  // order.
  if constexpr (UPD && !SP) {
    constexpr int NP = R * R;
    const int nct = n_pad / TC;
    const int npb = ct < NP ? (NP - ct + nct - 1) / nct : 0;   // pairs of this tile
    double* gbuf = reinterpret_cast<double*>(tileP);
    const int nsr = nblocks * RB;   // rows of the slice
    for (int base = 0; base < npb; base += 256) {
      const int cnt = npb - base < 256 ? npb - base : 256;
      const int G = 256 / cnt;
      const int pi = tid % cnt, grp = tid / cnt;
      const int pair = ct + nct * (base + pi);
      __syncthreads();
      double g = 0.0;
      if (grp < G) {
        const int a = pair / R, bb = pair % R;
        const T* vp = Vj + a;
        const T* up = Uj + bb;
#pragma unroll 8
        for (int q = grp; q < nsr; q += G) {
          const int64_t i = blk_row(q / RB) + q % RB;
          g = fma((double)vp[i * W], (double)up[i * W], g);
        }
      }
      gbuf[tid] = g;
      __syncthreads();
      if (tid < cnt) {
        double sum = 0.0;
        for (int q = 0; q < G; ++q) sum += gbuf[q * cnt + tid];
        partG[(int64_t)rt * NP + pair] = sum;
      }
    }
  }
}

template <typename T, int R, int RB, bool UPD>
__global__ void __launch_bounds__(256) k_level_fused(const FusedDesc<T> d) {
  fused_body<T, R, RB, UPD>(d.P, d.ldp, d.n_pad, d.tile_rows, d.Uj, d.Vj, d.W, d.partX, d.partY, d.partG, d.pR,
                            blockIdx.x, blockIdx.y);
}

// The same pass with gridDim.y below the slice count: row slices rt =
// blockIdx.y, blockIdx.y + gridDim.y, ... one after the other (fewer,
// longer-lived work-groups; every slice is summed exactly as with one
// work-group per slice, so the partials are the same bit for bit).
template <typename T, int R, int RB, bool UPD>
__global__ void __launch_bounds__(256) k_level_fused_grouped(const FusedDesc<T> d) {
  const int ns = (d.n_pad + d.tile_rows - 1) / d.tile_rows;
  for (int rt = blockIdx.y; rt < ns; rt += gridDim.y) {
    fused_body<T, R, RB, UPD>(d.P, d.ldp, d.n_pad, d.tile_rows, d.Uj, d.Vj, d.W, d.partX, d.partY, d.partG, d.pR,
                              blockIdx.x, rt);
    __syncthreads();   // the next slice restages the LDS tiles
  }
}

// The powers' pass of a view with sums or a general form: X also for Q_j
// (XE = R columns or none) and for D_j (XD columns or none).
template <typename T, int R, int RB, int XE, int XD>
__global__ void __launch_bounds__(256) k_level_fused_x(const FusedDesc<T> d) {
  fused_body<T, R, RB, true, XE, false, XD>(d.P, d.ldp, d.n_pad, d.tile_rows, d.Uj, d.Vj, d.W, d.partX, d.partY,
                                            d.partG, d.pR, blockIdx.x, blockIdx.y, d.Ux, d.partX2, nullptr, d.Ud,
                                            d.Wd, d.partX3);
}

// The sums pass: Y = S^T Vy (old S), S += Q_j W_j^T.
template <typename T, int R, int RB>
__global__ void __launch_bounds__(256) k_sums_fused(const FusedDesc<T> d) {
  fused_body<T, R, RB, true, 0, true>(d.P, d.ldp, d.n_pad, d.tile_rows, d.Uj, d.Vj, d.W, nullptr, d.partY, nullptr,
                                      d.pR, blockIdx.x, blockIdx.y, nullptr, nullptr, d.Vy);
}

template <typename T, int R, int RB, bool UPD>
__global__ void __launch_bounds__(256) k_level_fused_multi(const FusedDesc<T>* __restrict__ ds, int nd) {
  const int v = find_desc(ds, nd, (int)blockIdx.x);
  const FusedDesc<T> d = load_desc(ds, v);
  const int local = (int)blockIdx.x - d.block_begin;
  fused_body<T, R, RB, UPD>(d.P, d.ldp, d.n_pad, d.tile_rows, d.Uj, d.Vj, d.W, d.partX, d.partY, d.partG, d.pR,
                            local % d.nct, local / d.nct);
}

template <typename T, int R, int RB, bool UPD>
hipError_t fused_launch(T* P, int64_t ldp, int64_t n_pad, int tile_rows, const T* Uj, const T* Vj,
                        int W, T* partX, T* partY, double* partG, int pR, hipStream_t s, int slice_groups = 0) {
  const int nct = (int)(n_pad / tile_cols<T>());
  const FusedDesc<T> d{P, ldp, (int)n_pad, tile_rows, Uj, Vj, W, partX, partY, partG, pR, nct, 0};
  const int ns = (int)((n_pad + tile_rows - 1) / tile_rows);
  if constexpr (UPD && R <= 8) {
    if (slice_groups > 0 && slice_groups < ns) {
      hipLaunchKernelGGL((k_level_fused_grouped<T, R, RB, UPD>), dim3((unsigned)nct, (unsigned)slice_groups),
                         dim3(256), 0, s, d);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_level_fused<T, R, RB, UPD>), dim3((unsigned)nct, (unsigned)ns), dim3(256), 0, s, d);
  return hipGetLastError();
}

// One level with rank R: for R <= 16 the fused pass; above, the skinny
// products in 16-column chunks (read-only passes), the Gram, then the rank-R
// update pass.
template <typename T, int R>
hipError_t fused_r(T* P, int64_t ldp, int64_t n_pad, int tile_rows, const T* Uj, const T* Vj,
                   int W, T* partX, T* partY, double* partG, hipStream_t s, int slice_groups) {
  if constexpr (R <= kMaxFusedRank) {
    constexpr int RB = fused_row_block(R);
    return fused_launch<T, R, RB, true>(P, ldp, n_pad, tile_rows, Uj, Vj, W, partX, partY, partG, R, s,
                                        slice_groups);
  } else {
    constexpr int RC = kMaxFusedRank;
    for (int c0 = 0; c0 < R; c0 += RC) {
      hipError_t e = fused_launch<T, RC, 8, false>(P, ldp, n_pad, tile_rows, Uj + c0, Vj + c0, W,
                                                   partX + c0, partY + c0, nullptr, R, s);
      if (e != hipSuccess) return e;
    }
    const T* slabV = Vj - (W - R);
    hipError_t e = launch_level_gram<T>(R, Uj, slabV, W, n_pad, partG, s);
    if (e != hipSuccess) return e;
    return launch_level_update<T>(R, P, ldp, n_pad, Uj, slabV, W, s);
  }
}

}  // namespace

template <typename T>
hipError_t launch_level_fused(int R, T* P, int64_t ldp, int64_t n_pad, int tile_rows,
                              const T* slabU, const T* slabV, int W, T* partX, T* partY,
                              double* partG, hipStream_t s, int slice_groups) {
  const T* Uj = slabU;
  const T* Vj = slabV + (W - R);
  LV_RANK_SWITCH(R, return (fused_r<T, RR>(P, ldp, n_pad, tile_rows, Uj, Vj, W, partX, partY, partG, s,
                                           slice_groups)))
}

// Launch k_level_fused_x for level rank R with XE (0 or R) and xd (0, 1, 2,
// 4 or 8) extra columns, R + XE + xd <= fused_x_cap(R); the row blocks (RB) of the plain
// pass for the same R: the same summation order, so X for U_j, Y, the Gram
// and the update are bit-identical to it.
template <typename T, int R, int XE>
hipError_t fused_x_launch(int xd, const FusedDesc<T>& d, dim3 grid, hipStream_t s) {
  constexpr int RB = fused_row_block(R);
  switch (xd) {
#define LV_FUSED_X_CASE(XD)                                                                   \
    case XD:                                                                                  \
      if constexpr (R + XE + XD <= fused_x_cap(R)) {                                          \
        hipLaunchKernelGGL((k_level_fused_x<T, R, RB, XE, XD>), grid, dim3(256), 0, s, d);    \
        return hipGetLastError();                                                             \
      }                                                                                       \
      return hipErrorInvalidValue;
    LV_FUSED_X_CASE(0)
    LV_FUSED_X_CASE(1)
    LV_FUSED_X_CASE(2)
    LV_FUSED_X_CASE(4)
    LV_FUSED_X_CASE(8)
#undef LV_FUSED_X_CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_level_fused_x(int R, T* P, int64_t ldp, int64_t n_pad, int tile_rows, const T* slabU,
                                const T* slabV, int W, T* partX, T* partY, double* partG, const T* slabQ, T* partXq,
                                const T* Dop, int ldd, int xd, T* partXd, hipStream_t s) {
  if (!fused_extra_fits(R, slabQ != nullptr, xd)) return hipErrorInvalidValue;
  const int nct = (int)(n_pad / tile_cols<T>());
  FusedDesc<T> d{P, ldp, (int)n_pad, tile_rows, slabU, slabV + (W - R), W, partX, partY, partG, R, nct, 0};
  d.Ux = slabQ;
  d.partX2 = partXq;
  d.Ud = Dop;
  d.Wd = ldd;
  d.partX3 = partXd;
  const dim3 grid((unsigned)nct, (unsigned)((n_pad + tile_rows - 1) / tile_rows));
  const bool q = slabQ != nullptr;
  switch (R) {
    case 1: return q ? fused_x_launch<T, 1, 1>(xd, d, grid, s) : fused_x_launch<T, 1, 0>(xd, d, grid, s);
    case 2: return q ? fused_x_launch<T, 2, 2>(xd, d, grid, s) : fused_x_launch<T, 2, 0>(xd, d, grid, s);
    case 4: return q ? fused_x_launch<T, 4, 4>(xd, d, grid, s) : fused_x_launch<T, 4, 0>(xd, d, grid, s);
    case 8: return q ? fused_x_launch<T, 8, 8>(xd, d, grid, s) : fused_x_launch<T, 8, 0>(xd, d, grid, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_sums_fused(int R, T* S, int64_t ldp, int64_t n_pad, int tile_rows, const T* slabQ,
                             const T* slabW, const T* slabV, int W, T* partY, hipStream_t s) {
  const int nct = (int)(n_pad / tile_cols<T>());
  FusedDesc<T> d{S, ldp, (int)n_pad, tile_rows, slabQ, slabW + (W - R), W, nullptr, partY, nullptr, R, nct, 0};
  d.Vy = slabV + (W - R);
  const dim3 grid((unsigned)nct, (unsigned)((n_pad + tile_rows - 1) / tile_rows));
  switch (R) {
    case 1: hipLaunchKernelGGL((k_sums_fused<T, 1, 8>), grid, dim3(256), 0, s, d); break;
    case 2: hipLaunchKernelGGL((k_sums_fused<T, 2, 8>), grid, dim3(256), 0, s, d); break;
    case 4: hipLaunchKernelGGL((k_sums_fused<T, 4, 8>), grid, dim3(256), 0, s, d); break;
    case 8: hipLaunchKernelGGL((k_sums_fused<T, 8, 8>), grid, dim3(256), 0, s, d); break;
    case 16: hipLaunchKernelGGL((k_sums_fused<T, 16, 8>), grid, dim3(256), 0, s, d); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fused_multi(int R, bool chunk, const FusedDesc<T>* ds, int nd, int blocks, hipStream_t s) {
  if (blocks <= 0) return hipSuccess;
  if (chunk) {
    hipLaunchKernelGGL((k_level_fused_multi<T, kMaxFusedRank, 8, false>), dim3((unsigned)blocks), dim3(256), 0, s,
                       ds, nd);
    return hipGetLastError();
  }
  switch (R) {
    case 1: hipLaunchKernelGGL((k_level_fused_multi<T, 1, fused_row_block(1), true>), dim3((unsigned)blocks), dim3(256), 0, s, ds, nd); break;
    case 2: hipLaunchKernelGGL((k_level_fused_multi<T, 2, fused_row_block(2), true>), dim3((unsigned)blocks), dim3(256), 0, s, ds, nd); break;
    case 4: hipLaunchKernelGGL((k_level_fused_multi<T, 4, fused_row_block(4), true>), dim3((unsigned)blocks), dim3(256), 0, s, ds, nd); break;
    case 8: hipLaunchKernelGGL((k_level_fused_multi<T, 8, fused_row_block(8), true>), dim3((unsigned)blocks), dim3(256), 0, s, ds, nd); break;
    case 16: hipLaunchKernelGGL((k_level_fused_multi<T, 16, fused_row_block(16), true>), dim3((unsigned)blocks), dim3(256), 0, s, ds, nd); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Read-only pass: partial X = P Uop and Y = P^T Vop for R columns (row
// stride R), P unchanged: the fused kernel without its update and Gram, in
// 16-column chunks above 16.
template <typename T>
hipError_t launch_level_readonly(int R, const T* P, int64_t ldp, int64_t n_pad, int tile_rows, const T* Uop,
                                 const T* Vop, int W, T* partX, T* partY, hipStream_t s) {
  T* Pm = const_cast<T*>(P);   // not written: UPD = false
  switch (R) {
    case 1: return fused_launch<T, 1, fused_row_block(1), false>(Pm, ldp, n_pad, tile_rows, Uop, Vop, W, partX, partY, nullptr, R, s);
    case 2: return fused_launch<T, 2, fused_row_block(2), false>(Pm, ldp, n_pad, tile_rows, Uop, Vop, W, partX, partY, nullptr, R, s);
    case 4: return fused_launch<T, 4, fused_row_block(4), false>(Pm, ldp, n_pad, tile_rows, Uop, Vop, W, partX, partY, nullptr, R, s);
    case 8: return fused_launch<T, 8, fused_row_block(8), false>(Pm, ldp, n_pad, tile_rows, Uop, Vop, W, partX, partY, nullptr, R, s);
    default: break;
  }
  if (R % kMaxFusedRank != 0 || R > 128) return hipErrorInvalidValue;
  for (int c0 = 0; c0 < R; c0 += kMaxFusedRank) {
    const hipError_t e = fused_launch<T, kMaxFusedRank, 8, false>(Pm, ldp, n_pad, tile_rows, Uop + c0, Vop + c0, W,
                                                                  partX + c0, partY + c0, nullptr, R, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t launch_level_readonly<float>(int, const float*, int64_t, int64_t, int, const float*, const float*,
                                                 int, float*, float*, hipStream_t);
template hipError_t launch_level_readonly<double>(int, const double*, int64_t, int64_t, int, const double*,
                                                  const double*, int, double*, double*, hipStream_t);

template hipError_t launch_level_fused<float>(int, float*, int64_t, int64_t, int, const float*, const float*, int,
                                              float*, float*, double*, hipStream_t, int);
template hipError_t launch_level_fused<double>(int, double*, int64_t, int64_t, int, const double*, const double*,
                                               int, double*, double*, double*, hipStream_t, int);
template hipError_t launch_level_fused_x<float>(int, float*, int64_t, int64_t, int, const float*, const float*, int,
                                                float*, float*, double*, const float*, float*, const float*, int, int,
                                                float*, hipStream_t);
template hipError_t launch_level_fused_x<double>(int, double*, int64_t, int64_t, int, const double*, const double*,
                                                 int, double*, double*, double*, const double*, double*,
                                                 const double*, int, int, double*, hipStream_t);
template hipError_t launch_sums_fused<float>(int, float*, int64_t, int64_t, int, const float*, const float*,
                                             const float*, int, float*, hipStream_t);
template hipError_t launch_sums_fused<double>(int, double*, int64_t, int64_t, int, const double*, const double*,
                                              const double*, int, double*, hipStream_t);
template hipError_t launch_fused_multi<float>(int, bool, const FusedDesc<float>*, int, int, hipStream_t);
template hipError_t launch_fused_multi<double>(int, bool, const FusedDesc<double>*, int, int, hipStream_t);

}  // namespace lv
