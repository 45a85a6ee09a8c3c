// Internal declarations shared by the HIP translation units of liblinview.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace lv {

// Every stored power is padded to a multiple of this order; the padding
// rows and columns hold zeros and stay zero under every operation (a zero
// row of P_j or U_j produces zero rows of every product), so no kernel needs
// bounds checks.
constexpr int kPadOrder = 256;
// A tile's row count and the padded order are multiples of 4 waves x 16-row
// blocks in the fused level pass.
// Largest level rank handled by the register-resident fused pass; larger
// ranks run the skinny products in chunks of this many factor columns.
constexpr int kMaxFusedRank = 16;
// Rows per block of the fused level pass for level rank R: a wave streams
// RB rows of its 16-byte column group per step.
constexpr int fused_row_block(int R) { return R >= 8 ? 8 : 4; }
// Row blocks of the fused pass in flight beyond the one being processed.
constexpr int fused_prefetch(int R) { return R >= 8 ? 0 : 1; }
// Largest level of the exponential model (k <= 2^kMaxLevel).
constexpr int kMaxLevel = 10;
// Pipelined batches: at most this many stage streams and factor-slab slots
// (updates in flight).
constexpr int kPipeStreams = 4;
constexpr int kMaxPipeSlots = 5;
// Work-groups a fused level pass is cut into inside a pipelined batch: one
// per compute unit (the device has 256), so that the passes of two stages
// share every unit instead of one pass filling the device with two
// work-groups per unit.  Returns the work-groups per column tile for nct
// column tiles and ns row slices (each takes ceil(ns / groups) slices;
// never fewer than kPipePassBlocks work-groups in all).
constexpr int kPipePassBlocks = 256;
inline int pipe_slice_groups(int nct, int ns) {
  const int spb = nct * ns / kPipePassBlocks;
  return spb <= 1 ? ns : (ns + spb - 1) / spb;
}

inline int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// float -> bfloat16 bits, rounding to nearest even (v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint16_t bf16_rne(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }

// Columns covered by one tile of the level pass: a wave reads a 1 KiB row
// segment with one 16-byte vector per lane.
template <typename T> constexpr int tile_cols() { return 64 * (16 / (int)sizeof(T)); }
inline int tile_cols_bytes(int elem) { return 64 * (16 / elem); }

// ---- work descriptors ----
// One descriptor per (view, kernel) in a launch.  A single-view launch passes
// one descriptor by value; a multi-view launch passes a device array sorted
// by block_begin (the first work-group of each view) and the work-group
// finds its view by binary search.

template <typename T> struct FusedDesc {
  T* P; int64_t ldp; int n_pad; int tile_rows;
  const T* Uj; const T* Vj; int W;      // U_j = Uj[i*W + c], V_j = Vj[i*W + c]
  T* partX; T* partY; double* partG; int pR;
  int nct; int block_begin;             // blocks: nct x ceil(n_pad / tile_rows)
  const T* Ux = nullptr;                // extra X operand (powers' pass of a view with sums)
  T* partX2 = nullptr;                  //   and its partials
  const T* Vy = nullptr;                // Y operand of the sums pass
  const T* Ud = nullptr; int Wd = 0;    // general form: extra X operand (row stride Wd)
  T* partX3 = nullptr;                  //   and its partials
};
template <typename T> struct GramDesc {
  const T* Uj; const T* Vj; int W; int n_pad; int tile_rows; double* partG;
  int nrt; int block_begin;             // blocks: nrt x pair chunks
};
template <typename T> struct TailDesc {
  const T* partX; const T* partY; const double* partG; int nct; int nrt; int n_pad;
  T* slabU; T* slabV; int W; int block_begin;   // blocks: ceil(n_pad * R / 256)
  int ng;                                       // Gram partials to add (1: already summed)
};
// Sum of ng Gram partials (count doubles each) into the first.
struct GramSumDesc {
  double* G; int ng; int count; int block_begin;   // blocks: ceil(count / 256)
};
template <typename T> struct UpdateDesc {
  T* P; int64_t ldp; int n_pad; int tile_rows; const T* Uj; const T* Vj; int W;
  int nct; int block_begin;             // blocks: nct x ceil(n_pad / tile_rows)
  uint16_t* S;                          // bfloat16 shadow of P rewritten by the pass, or null
};
// Products a read-only skinny pass forms.
constexpr int kWantX = 1, kWantY = 2;
// Read-only skinny products of a level on the matrix cores, from the
// bfloat16 shadow of P or from P itself (float): X = P U_j and Y = P^T V_j
// for R columns of the factors (partials with row stride pR, as FusedDesc).
struct SkinnyDesc {
  const void* src; int64_t ldp; int n_pad; int tile_rows;
  const float* Uj; const float* Vj; int W; int R;
  float* partX; float* partY; int pR;
  int nct; int block_begin;             // blocks: nct x ceil(n_pad / tile_rows)
  int want = kWantX | kWantY;           // products formed (float pass only)
};
template <typename T> struct PrepDesc {
  const T* U; int64_t ldu; const T* V; int64_t ldv; int64_t n; int r; int r_pad;
  T* slabU; T* slabV; int W; int64_t n_pad; int block_begin;   // blocks: ceil(n_pad * r_pad / 256)
};

// Descriptor v of a multi-view launch, read through the constant address
// space.  The table is written by the host before the launch and only read
// by it, and the compiler takes pointers loaded from constant memory to
// address global memory: accesses through the descriptor's pointers are then
// global instructions.  Read as ordinary (generic) memory, the pointers would
// be generic too, and their flat accesses count against the LDS wait counter
// as well, so that every wait for an LDS read would also wait for the HBM
// loads in flight.
// (The host pass of the compiler, which only declares the kernels, has no
// address space 4.)
template <typename D> __device__ __forceinline__ D load_desc(const D* ds, int v) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *((const __attribute__((address_space(4))) D*)ds + v);
#else
  return ds[v];
#endif
}

// Tiling of the update pass.  The vector kernel covers tiles of 256 rows x
// (64 lanes x 16 bytes); float storage with rank R >= kMfmaUpdateRank uses
// the matrix-core kernel on 128 x 128 tiles.
constexpr int kUpdateTileRows = 256;
// Level ranks of a plain view run up to kMaxLevelRank (the factors of the
// level below the top; LV_RANK_SWITCH covers 1 .. kMaxLevelRank / 2), the
// top update up to twice that.
constexpr int kMaxLevelRank = 256;
constexpr int kMfmaUpdateRank = 32;
constexpr int kMfmaUpdateTile = 128;
inline bool update_on_mfma(int R, int elem) { return elem == 4 && R >= kMfmaUpdateRank; }
inline int update_tile_rows(int R, int elem) { return update_on_mfma(R, elem) ? kMfmaUpdateTile : kUpdateTileRows; }
// Work-groups a single-view streaming pass aims for, and the rows per
// (interleaved) slice of the vector update pass that give about that many
// for one view of padded order n_pad (several views in one launch keep
// update_tile_rows).
constexpr int kStreamBlocks = 512;
inline int update_slice_rows(int R, int elem, int64_t n_pad) {
  if (update_on_mfma(R, elem)) return kMfmaUpdateTile;
  const int64_t nct = n_pad / tile_cols_bytes(elem);
  int64_t ns = kStreamBlocks / (nct > 0 ? nct : 1);
  const int64_t ns_max = n_pad / (4 * 8);   // at least one 8-row block per wave
  ns = ns < 1 ? 1 : ns > ns_max ? ns_max : ns;
  return (int)((n_pad + ns - 1) / ns);
}
inline int update_tile_cols(int R, int elem) { return update_on_mfma(R, elem) ? kMfmaUpdateTile : tile_cols_bytes(elem); }
// Rows per partial of the stand-alone Gram kernel, and its partial count.
constexpr int kGramRows = 64;
inline int gram_tiles(int64_t n_pad) { return (int)(n_pad / kGramRows); }
// Float storage with level rank R >= kMfmaSkinnyRank forms the skinny
// products on the matrix cores in a read-only pass (then Gram, update);
// smaller ranks use the fused vector pass.
constexpr int kMfmaSkinnyRank = 16;
inline bool skinny_on_mfma(int R, int elem) { return elem == 4 && R >= kMfmaSkinnyRank; }
// Whether the fused pass of rank R forms the Gram partials itself (one per
// row tile); otherwise the stand-alone Gram kernel and its sum provide G.
inline bool gram_in_pass(int R, int elem) { return R <= kMaxFusedRank && !skinny_on_mfma(R, elem); }
// The powers' fused pass of a level with rank R can also form X for Q_j (R
// more columns, views with sums) and for xd columns of a general-form operand
// (xd a power of two up to 8) when the level runs the fused vector pass and
// the X width stays within fused_x_cap(R): 16 columns with the 8-row blocks
// of R = 8, 12 with the 16-row blocks below (the LDS of two blocks per CU).
constexpr int fused_x_cap(int R) { return R >= 8 ? 16 : 12; }
inline bool fused_extra_fits(int R, bool q, int xd) {
  return R <= 8 && (xd == 0 || xd == 1 || xd == 2 || xd == 4 || xd == 8) && R + (q ? R : 0) + xd <= fused_x_cap(R);
}
inline bool fused_vector_level(int R, int elem, bool shadowed) { return !shadowed && !skinny_on_mfma(R, elem); }
// The sums pass (Y = S^T V_j and the rank update of S in one pass) on the
// vector kernel, below the ranks that run on the matrix cores.
inline bool sums_fused(int R, int elem) { return R <= kMaxFusedRank && !skinny_on_mfma(R, elem); }
// Work-groups of a tail launch / Gram pairs per work-group for rank R.
// Level ranks from which the tail works on column slices of min(R, 32)
// columns, one column per lane and kTailRowsPerThread rows per thread.
constexpr int kSlicedTailRank = 16;
constexpr int kTailRowsPerThread = 4;
inline int tail_slice_cols(int R) { return R < 32 ? R : 32; }
inline int tail_block_rows(int R) { return 256 / tail_slice_cols(R) * kTailRowsPerThread; }
// Lanes per output entry of the tail below kSlicedTailRank.
constexpr int kTailLanes = 8;
inline int tail_blocks(int64_t n_pad, int R) {
  return R >= kSlicedTailRank ? (int)(n_pad / tail_block_rows(R)) * (R / tail_slice_cols(R))
                              : (int)((n_pad * R * kTailLanes + 255) / 256);
}
inline int gram_pairs_per_block(int R) {
  const int ppt = (R * R + 255) / 256 < 16 ? (R * R + 255) / 256 : 16;
  return 256 * ppt;
}

// ---- launchers (stream-ordered; return the launch status) ----

// dst[i*ldd + j] = (i < n && j < n) ? src[i*lds + j] : 0 for i, j < n_pad.
// With a non-null `gate`, the kernel does nothing unless *gate != 0 (read on
// the device, so a decision taken by an earlier kernel needs no host sync).
template <typename Tin, typename Tout>
hipError_t launch_copy_pad(const Tin* src, int64_t lds, int64_t n, Tout* dst, int64_t ldd,
                           int64_t n_pad, hipStream_t s, const int* gate = nullptr);

// Factor slab set-up: slab U columns [0, r_pad) and slab V columns
// [W - r_pad, W) receive U and V (n x r), zero-filled up to r_pad columns and
// n_pad rows.
template <typename T>
hipError_t launch_prep(const T* U, int64_t ldu, const T* V, int64_t ldv, int64_t n, int r,
                       int r_pad, T* slabU, T* slabV, int W, int64_t n_pad, hipStream_t s);

// Fused level pass for level rank R: partial X = P U_j, partial Y = P^T V_j,
// partial Gram V_j^T U_j (column tile 0 only), and P += U_j V_j^T, in one
// read and one write of P.  slice_groups > 0: that many work-groups per
// column tile, each taking several row slices in turn (same partials, bit
// for bit; see pipe_slice_groups).
template <typename T>
hipError_t launch_level_fused(int R, T* P, int64_t ldp, int64_t n_pad, int tile_rows,
                              const T* slabU, const T* slabV, int W, T* partX, T* partY,
                              double* partG, hipStream_t s, int slice_groups = 0);

// Tail of level j: reduce partials in a fixed order, G = sum of the ng
// partial Grams, U_{j+1} = [U_j, X + U_j G], V_{j+1} = [Y, V_j].
template <typename T>
hipError_t launch_level_tail(int R, const T* partX, const T* partY, const double* partG,
                             int nct, int nrt, int ng, int64_t n_pad, T* slabU, T* slabV, int W,
                             hipStream_t s);

// Update-only pass: P += U_j V_j^T for rank R (the top stored power).  With a
// non-null shadow S (float only) the pass also writes S = bf16(P) of the new
// values.  `split` (float, bfloat16-shadow mode) forms the matrix-core ranks
// with split bfloat16 operands (three products) instead of float products.
template <typename T>
hipError_t launch_level_update(int R, T* P, int64_t ldp, int64_t n_pad, const T* slabU,
                               const T* slabV, int W, hipStream_t s, uint16_t* S = nullptr,
                               bool split = false);

// Gram V_j^T U_j in double: gram_tiles(n_pad) partials of kGramRows rows,
// then their sum in fixed order into partG[0 .. R*R).
template <typename T>
hipError_t launch_level_gram(int R, const T* slabU, const T* slabV, int W, int64_t n_pad, double* partG,
                             hipStream_t s);
hipError_t launch_gram_sum_multi(const GramSumDesc* ds, int nd, int blocks, hipStream_t s);

// Skinny products of level rank R (<= kMaxLevelRank) from the bfloat16 shadow S on the
// matrix cores (bf16 x bf16 -> fp32): partial X = S U_j, partial Y = S^T V_j
// over tiles of tile_rows x 256 (partials as for the fused pass, row stride R).
hipError_t launch_skinny_bf16(int R, const uint16_t* S, int64_t ldp, int64_t n_pad, int tile_rows,
                              const float* slabU, const float* slabV, int W, float* partX, float* partY,
                              hipStream_t s);
hipError_t launch_skinny_bf16_multi(int nb, const SkinnyDesc* ds, int nd, int blocks, hipStream_t s);
// Factor blocks of 32 columns the bfloat16 skinny kernel needs for rank R.
inline int skinny_blocks_for(int R) { return R <= 32 ? 1 : 2; }   // R <= 64 per launch

// The same products from the float power P (v_mfma_f32_32x32x2f32, float
// products and accumulation), R <= kMaxLevelRank (32 factor columns per launch; X alone: 64).
// update: also apply P += U_j V_j^T in the same pass (one read and one write
// of P; R = 16 or 32, X and Y both, see skinny_fuses_update).
hipError_t launch_skinny_f32(int R, const float* P, int64_t ldp, int64_t n_pad, int tile_rows,
                             const float* slabU, const float* slabV, int W, float* partX, float* partY,
                             hipStream_t s, int want = kWantX | kWantY, bool update = false);
// nb: the width class below, plus 2 for the update-fused kernels.
hipError_t launch_skinny_f32_multi(int nb, const SkinnyDesc* ds, int nd, int blocks, hipStream_t s);
// Width class of a float skinny launch of at most 32 factor columns (0: the
// 16-wide pass for R <= 16; 1: one 32-column factor block).
inline int skinny_f32_blocks(int R) { return R <= 16 ? 0 : 1; }
// Float level ranks whose skinny pass on the matrix cores also applies the
// rank update (a second pass over P would otherwise follow).  The kernels
// take R = 16 or 32; at 32 the fused block (one per CU by its LDS, one
// 32-row chunk in flight) is slower than the skinny pass plus the update
// pass (839 vs 771 us at n = 16384), so only R = 16 uses it.
inline bool skinny_fuses_update(int R) { return R == 16; }
inline bool skinny_update_kernel(int R) { return R == 16 || R == 32; }

// S = bf16(P) for `count` consecutive floats (count a multiple of 4); with a
// non-null gate only when *gate != 0.
hipError_t launch_to_bf16(const float* P, uint16_t* S, int64_t count, hipStream_t s,
                          const int* gate = nullptr);

// ---- sums of powers (views with LV_WITH_SUMS)

// Read-only pass: partial X = P Uop, Y = P^T Vop for R columns (row stride
// R), P unchanged (fused kernel without its update).
template <typename T>
hipError_t launch_level_readonly(int R, const T* P, int64_t ldp, int64_t n_pad, int tile_rows, const T* Uop,
                                 const T* Vop, int W, T* partX, T* partY, hipStream_t s);
// The powers' fused pass with extra X columns (fused_extra_fits): as
// launch_level_fused for level rank R, and in the same read of P
// X = P Q_j (slabQ non-null; Q_j = columns [0, R) of slabQ, partials to
// partXq, [nct][n_pad][R]) and X = P D (Dop non-null; xd columns with row
// stride ldd, partials to partXd, [nct][n_pad][xd]).
template <typename T>
hipError_t launch_level_fused_x(int R, T* P, int64_t ldp, int64_t n_pad, int tile_rows, const T* slabU,
                                const T* slabV, int W, T* partX, T* partY, double* partG, const T* slabQ, T* partXq,
                                const T* Dop, int ldd, int xd, T* partXd, hipStream_t s);
// The sums pass (R <= 16): partial Y = S^T V_j with the old S (V_j = columns
// [W - R, W) of slabV; partials [nrt][n_pad][R]) and S += Q_j W_j^T, one read
// and one write of S.
template <typename T>
hipError_t launch_sums_fused(int R, T* S, int64_t ldp, int64_t n_pad, int tile_rows, const T* slabQ,
                             const T* slabW, const T* slabV, int W, T* partY, hipStream_t s);
// G = Vop^T Uop (R x R, double) into partG[0 .. R*R), operands given by
// their first columns (row stride W).
template <typename T>
hipError_t launch_gram_cols(int R, const T* Uop, const T* Vop, int W, int64_t n_pad, double* partG, hipStream_t s);
// Factors of the next level's sums (see k_sums_tail): Q_{j+1} = [U_j, X + Q_j],
// W_{j+1} = [Y + W_j G, W_j]; `first` for level 0 (Q_0 = 0, S_0 = I).
template <typename T>
hipError_t launch_sums_tail(int R, const T* partX, const T* partY, const double* G, int nct, int nrt, int64_t n_pad,
                            T* slabQ, T* slabW, const T* slabU, const T* slabV, int W, bool first, hipStream_t s);
// S = I (n x n identity, zero padding to n_pad); dst += src (count elements).
// With a non-null gate only when *gate != 0.
template <typename T>
hipError_t launch_set_identity(T* S, int64_t ld, int64_t n, int64_t n_pad, hipStream_t s, const int* gate = nullptr);
template <typename T>
hipError_t launch_add(T* dst, const T* src, int64_t count, hipStream_t s, const int* gate = nullptr);

// ---- general form T_{i+1} = A T_i + B (hybrid deltas)

// part[0 .. R*p) = A^T B (double) for A n_pad x R (lda), B n_pad x p (ldb):
// 64-row partials, then their fixed-order sum (part holds n_pad / 64 partials).
template <typename T>
hipError_t launch_atb(int R, int p, const T* A, int64_t lda, const T* B, int64_t ldb, int64_t n_pad, double* part,
                      hipStream_t s);
// D = sum of nct partials of X + U a (+ Q b if Q is non-null), T += D
// (n_pad x pp; U, Q with row stride W and R columns; a, b R x pp double).
template <typename T>
hipError_t launch_general_tail(const T* partX, int nct, const T* U, const T* Q, int W, int R, const double* a,
                               const double* b, T* D, T* Tm, int64_t n_pad, int pp, hipStream_t s);
// C = A B (+ C0 if non-null), A n_pad x n_pad (lda), B, C, C0 n_pad x pp,
// double; pp in {1, 2, 4, ..., 64}.  With a non-null gate only when *gate != 0.
hipError_t launch_gemm_np(int pp, const double* A, int64_t lda, const double* B, double* C, const double* C0,
                          int64_t n_pad, hipStream_t s, const int* gate = nullptr);
// dst (n_pad x pp, contiguous) = src (n x p, ld lds) zero-padded.
template <typename Tin, typename Tout>
hipError_t launch_copy_rect(const Tin* src, int64_t lds, int64_t n, int p, Tout* dst, int64_t n_pad, int pp,
                            hipStream_t s, const int* gate = nullptr);
// Factored general-form deltas (Delta T_j = Y_j Z_j^T):
// Ynew (n_pad x WYn) = [U_j (R cols, row stride W), sum of nct partials of
// P_j Y_j (width wy, partial row stride pR) + U_j G (G R x ldg double),
// Q_j (R cols, stride W; zero if Q is null), 0 ...].
template <typename T>
hipError_t launch_gfac_y(const T* partX, int nct, int pR, const T* U, const T* Q, int W, int R, const double* G,
                         int ldg, int wy, T* Ynew, int WYn, int64_t n_pad, hipStream_t s);
// Ztnew (WYn x pp, factor-major) = [a (R x pp, double), Zt_j (wy rows),
// b (R x pp, double; zero if null), 0 ...].
template <typename T>
hipError_t launch_gfac_z(const double* a, const T* Zt, int wy, const double* b, int R, T* Ztnew, int WYn, int pp,
                         hipStream_t s);
// Tm (n_pad x pp) += Y (w columns, row stride sy) Zt (w x pp), double sums.
template <typename T>
hipError_t launch_rank_rect(T* Tm, const T* Y, int sy, const T* Zt, int w, int64_t n_pad, int pp, hipStream_t s);
// G[0 .. count) = sum over t < ng of G[t count + ...] (fixed order).
hipError_t launch_gram_sum(double* G, int ng, int count, hipStream_t s);

// Multi-view launches over device descriptor arrays (nd descriptors,
// `blocks` work-groups in total).  `chunk` selects the read-only skinny pass
// over 16 factor columns used for level ranks above kMaxFusedRank.
template <typename T>
hipError_t launch_fused_multi(int R, bool chunk, const FusedDesc<T>* ds, int nd, int blocks, hipStream_t s);
template <typename T>
hipError_t launch_gram_multi(int R, const GramDesc<T>* ds, int nd, int blocks, hipStream_t s);
template <typename T>
hipError_t launch_tail_multi(int R, const TailDesc<T>* ds, int nd, int blocks, hipStream_t s);
template <typename T>
hipError_t launch_update_multi(int R, bool shadow, bool split, const UpdateDesc<T>* ds, int nd, int blocks,
                               hipStream_t s);
template <typename T>
hipError_t launch_prep_multi(const PrepDesc<T>* ds, int nd, int blocks, hipStream_t s);

// C = A * B for n_pad x n_pad row-major matrices (n_pad a multiple of 256),
// on MFMA (double: 16x16x4 f64; float: 32x32x2 f32).
template <typename T>
hipError_t launch_gemm(const T* A, int64_t lda, const T* B, int64_t ldb, T* C, int64_t ldc,
                       int64_t n_pad, hipStream_t s, const int* gate = nullptr);
// C = A * B for A M x K, B K x N (M, N multiples of 128, K of 16), same kernel.
template <typename T>
hipError_t launch_gemm_rect(const T* A, int64_t lda, const T* B, int64_t ldb, T* C, int64_t ldc, int64_t M,
                            int64_t N, int64_t K, hipStream_t s, const int* gate = nullptr);

// ---- drift check (FP64 test of the stored chain P_{j+1} = P_j P_j)

// x = z zero-padded to n_pad (double).
hipError_t launch_vec_pad(const double* z, int64_t n, double* x, int64_t n_pad, hipStream_t s);
hipError_t launch_sign_vector(double* z, int64_t n, int64_t n_pad, unsigned long long seed, hipStream_t s);

// y = P x with double accumulation, P n_pad x n_pad (ld ldp) of type T.
template <typename T>
hipError_t launch_matvec(const T* P, int64_t ldp, int64_t n_pad, const double* x, double* y,
                         hipStream_t s);

// rho_j = max|Pz[j+1] - PPz[j]| / max|Pz[j+1]| for j < m (Pz, PPz: n_pad
// doubles per level); *gate = (some rho_j > tau or not finite); the
// counter is incremented when the gate opens.
hipError_t launch_drift_residual(const double* Pz, const double* PPz, int m, int64_t n_pad,
                                 double tau, double* residuals, int* gate,
                                 unsigned long long* counter, hipStream_t s);

}  // namespace lv
