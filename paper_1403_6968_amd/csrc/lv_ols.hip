// Ordinary least squares maintained under rank-1 changes of the data
// (Sec. 5.1 with the Sherman-Morrison formula of Sec. 4).  X is m x n, Y is
// m x p, Z = X^T X, W = Z^{-1}, beta = W X^T Y, and for Delta X = u v^T
//     Delta Z = p1 q1^T + p2 q2^T,  p1 = v, q1 = X^T u, p2 = X^T u + v (u^T u), q2 = v,
// W takes the two outer products in turn by Sherman-Morrison and
//     Delta beta = R S^T X^T Y + W v u^T Y + R S^T v u^T Y     (Delta W = R S^T).
// Every product with W uses the OLD W, so one read-only pass over W gives
// W [p1 p2 v] and W^T [q1 q2]; the second Sherman-Morrison step is then
// exact in vector form (W1 p2 = W p2 + r1 (s1^T p2), W1^T q2 = W^T q2 +
// s1 (r1^T q2)), and W takes one rank-2 update.  Per update: one read of W,
// one read and write of W, O(mn) for X^T u and X += u v^T (O(n) for a row
// change), O(np) for beta.  Creation forms X^T X and X^T Y in double and
// inverts by the Newton-Schulz iteration X <- X (2I - Z X) on the double
// matrix cores.
#include "linview.h"
#include "lv_device.h"
#include "lv_internal.h"
#include "lv_view_impl.h"

#include <new>

using namespace lv;

namespace lv {
namespace {

constexpr int kOlsMaxCols = 64;
constexpr int64_t kOlsMaxOrder = 32768;
constexpr int kRedBlocks = 1024;

// C[i][j] = sum_k A[k][i] B[k][j] in double: A K x M (lda), B K x N (ldb),
// C M x N (ldc); K a multiple of 32.  32 x 32 output tiles, k in steps of
// 32 staged in LDS.
template <typename T>
__global__ void __launch_bounds__(256)
k_tn_gemm(const T* __restrict__ A, int64_t lda, const T* __restrict__ B, int64_t ldb, double* __restrict__ C,
          int64_t ldc, int64_t K, int M, int N) {
  __shared__ double sa[32][33];
  __shared__ double sb[32][33];
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = 0; k0 < K; k0 += 32) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kk = ty + 8 * q;
      sa[kk][tx] = i0 + tx < M ? (double)A[(k0 + kk) * lda + i0 + tx] : 0.0;
      sb[kk][tx] = j0 + tx < N ? (double)B[(k0 + kk) * ldb + j0 + tx] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < 32; ++kk) {
      const double b = sb[kk][tx];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = fma(sa[kk][ty + 8 * q], b, acc[q]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = i0 + ty + 8 * q, j = j0 + tx;
    if (i < M && j < N) C[(int64_t)i * ldc + j] = acc[q];
  }
}

// Block-wide max of a per-thread value (256 threads), result in thread 0.
__device__ double block_max(double x) {
  __shared__ double red[256];
  red[threadIdx.x] = x;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  return red[0];
}

__device__ double block_sum(double x) {
  __shared__ double red[256];
  red[threadIdx.x] = x;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

// part[b] = max over this block's rows i < lim of sum_{j < lim} |Z[i][j]|
// (Z n_pad x n_pad).
__global__ void __launch_bounds__(256) k_rowabs_max(const double* __restrict__ Z, int64_t lim, int64_t n_pad,
                                                    double* part) {
  double best = 0.0;
  for (int64_t i = blockIdx.x; i < lim; i += gridDim.x) {
    double sacc = 0.0;
    for (int64_t j = threadIdx.x; j < lim; j += 256) sacc += fabs(Z[i * n_pad + j]);
    const double row = block_sum(sacc);
    best = fmax(best, row);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = best;
}

// out[0] = max of part[0 .. count) (one block).
__global__ void __launch_bounds__(256) k_max_reduce(const double* __restrict__ part, int count, double* out) {
  double best = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) best = fmax(best, part[i]);
  best = block_max(best);
  if (threadIdx.x == 0) out[0] = best;
}

// X = I / scale[0].
__global__ void __launch_bounds__(256) k_scaled_identity(double* __restrict__ X, int64_t n_pad, const double* scale) {
  const double a = 1.0 / scale[0];
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n_pad * n_pad; e += (int64_t)gridDim.x * 256)
    X[e] = (e / n_pad == e % n_pad) ? a : 0.0;
}

// Newton-Schulz step on T = Z X: part[b] = max |T - I| over the block's
// elements, then T = 2I - T.
__global__ void __launch_bounds__(256) k_ns_step(double* __restrict__ T, int64_t n_pad, double* part) {
  double best = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n_pad * n_pad; e += (int64_t)gridDim.x * 256) {
    const double id = (e / n_pad == e % n_pad) ? 1.0 : 0.0;
    const double d = T[e] - id;
    best = fmax(best, fabs(d));
    T[e] = id - d;
  }
  best = block_max(best);
  if (threadIdx.x == 0) part[blockIdx.x] = best;
}

// Z[i][i] = 1 for n <= i < n_pad (so that the padded Z is invertible);
// with zero = true instead W[i][j] = 0 wherever i >= n or j >= n.
__global__ void __launch_bounds__(256) k_pad_square(double* __restrict__ Z, int64_t n, int64_t n_pad, bool zero) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n_pad * n_pad; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / n_pad, j = e % n_pad;
    if (i < n && j < n) continue;
    Z[e] = zero ? 0.0 : (i == j ? 1.0 : 0.0);
  }
}

// Operand slabs of the read-only pass over W: P = [p1, p2, v, 0],
// Q = [q1, q2, 0, 0] with p1 = q2 = v, q1 = X^T u, p2 = X^T u + v (u^T u).
template <typename T>
__global__ void __launch_bounds__(256)
k_ols_operands(const double* __restrict__ xu, const double* __restrict__ uu, const T* __restrict__ v,
               T* __restrict__ Pk, T* __restrict__ Qk, int64_t n_pad) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n_pad) return;
  const double vj = (double)v[j], x = xu[j];
  Pk[j * 4 + 0] = (T)vj;
  Pk[j * 4 + 1] = (T)(x + vj * uu[0]);
  Pk[j * 4 + 2] = (T)vj;
  Pk[j * 4 + 3] = T(0);
  Qk[j * 4 + 0] = (T)x;
  Qk[j * 4 + 1] = (T)vj;
  Qk[j * 4 + 2] = T(0);
  Qk[j * 4 + 3] = T(0);
}

constexpr int kVecRows = 64;   // rows per block of k_ols_vectors (4 threads per row)

// The 4-element partial record of row j in tile t (16 bytes for float, two
// 16-byte loads for double).
template <typename T>
__device__ __forceinline__ void load4(const T* __restrict__ rec, double (&o)[4]) {
  if constexpr (sizeof(T) == 4) {
    const V16<float> a = ld16(reinterpret_cast<const float*>(rec));
    o[0] = a.v[0]; o[1] = a.v[1]; o[2] = a.v[2]; o[3] = a.v[3];
  } else {
    const V16<double> a = ld16(reinterpret_cast<const double*>(rec));
    const V16<double> b = ld16(reinterpret_cast<const double*>(rec) + 2);
    o[0] = a.v[0]; o[1] = a.v[1]; o[2] = b.v[0]; o[3] = b.v[1];
  }
}

// vec[j] = (a1, a2, wv, b1, b2): W p1, W p2, W v, W^T q1, W^T q2 from the
// pass's partials, and this block's partial sums of the four dot products
// q1^T a1, b1^T p2, a1^T q2, q2^T a2 (dpart[blk][4]).  Four threads per row
// each sum every fourth tile; the four sums are added in order (double).
template <typename T>
__global__ void __launch_bounds__(256)
k_ols_vectors(const T* __restrict__ partX, int nct, const T* __restrict__ partY, int nrt, int64_t n_pad,
              const T* __restrict__ Pk, const T* __restrict__ Qk, double* __restrict__ vec, double* __restrict__ dpart) {
  __shared__ double sx[5][256];
  __shared__ double red[4][kVecRows];
  const int lr = (int)threadIdx.x >> 2, q = (int)threadIdx.x & 3;
  const int64_t j = (int64_t)blockIdx.x * kVecRows + lr;      // n_pad is a multiple of 256
  double x0 = 0.0, x1 = 0.0, x2 = 0.0, y0 = 0.0, y1 = 0.0;
  for (int t = q; t < nct; t += 4) {
    double r[4];
    load4(partX + ((int64_t)t * n_pad + j) * 4, r);
    x0 += r[0]; x1 += r[1]; x2 += r[2];
  }
  for (int t = q; t < nrt; t += 4) {
    double r[4];
    load4(partY + ((int64_t)t * n_pad + j) * 4, r);
    y0 += r[0]; y1 += r[1];
  }
  sx[0][threadIdx.x] = x0; sx[1][threadIdx.x] = x1; sx[2][threadIdx.x] = x2;
  sx[3][threadIdx.x] = y0; sx[4][threadIdx.x] = y1;
  __syncthreads();
  if (threadIdx.x < kVecRows) {
    const int b = (int)threadIdx.x * 4;
    const int64_t jj = (int64_t)blockIdx.x * kVecRows + threadIdx.x;
    double o5[5];
#pragma unroll
    for (int e = 0; e < 5; ++e) o5[e] = ((sx[e][b] + sx[e][b + 1]) + sx[e][b + 2]) + sx[e][b + 3];
    double* o = vec + jj * 5;
#pragma unroll
    for (int e = 0; e < 5; ++e) o[e] = o5[e];
    const double q1 = (double)Qk[jj * 4 + 0], q2 = (double)Qk[jj * 4 + 1], p2 = (double)Pk[jj * 4 + 1];
    red[0][threadIdx.x] = q1 * o5[0];
    red[1][threadIdx.x] = o5[3] * p2;
    red[2][threadIdx.x] = o5[0] * q2;
    red[3][threadIdx.x] = q2 * o5[1];
  }
  __syncthreads();
  for (int w = kVecRows / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int e = 0; e < 4; ++e) red[e][threadIdx.x] += red[e][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) dpart[blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

// out[b] = sum over i < nblk of part[i * stride + b] for b = blockIdx.x:
// 256 threads sum strided subsets, then a fixed-order tree.
__global__ void __launch_bounds__(256) k_sum_partials(const double* __restrict__ part, int nblk, int stride,
                                                      double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) acc += part[(int64_t)i * stride + blockIdx.x];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Update factors R = [r1, r2], S = [s1, s2] of Delta W, with the dots
// d0 = q1^T W p1, d1 = s1^T p2, d2 = r1^T q2 / l1, d3 = q2^T W p2:
//   l1 = -1 / (1 + d0),  r1 = l1 W p1,  s1 = W^T q1,
//   W1 p2 = W p2 + r1 (s1^T p2) = W p2 + l1 W p1 d1,
//   W1^T q2 = W^T q2 + s1 (r1^T q2) = W^T q2 + l1 W^T q1 d2,
//   l2 = -1 / (1 + q2^T W1 p2) = -1 / (1 + d3 + l1 d2 d1),
//   r2 = l2 W1 p2,  s2 = W1^T q2;
// then this block's partials of S^T C (2 x pp) and S^T v (2) with the stored
// (rounded) S: spart[blk][e * pp + c], spart[blk][2 pp + e].
template <typename T>
__global__ void __launch_bounds__(256)
k_ols_rs(const double* __restrict__ vec, const double* __restrict__ dots, T* __restrict__ Rs,
         T* __restrict__ Ss, const T* __restrict__ C, const T* __restrict__ v, int pp, double* __restrict__ spart) {
  __shared__ double ls[2][256];
  __shared__ double red[2][256];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const double l1 = -1.0 / (1.0 + dots[0]);
  const double l2 = -1.0 / (1.0 + dots[3] + l1 * dots[2] * dots[1]);
  const double* o = vec + j * 5;
  const double w1p2 = o[1] + l1 * o[0] * dots[1];
  const double w1q2 = o[4] + l1 * o[3] * dots[2];
  const T s1 = (T)o[3], s2 = (T)w1q2;
  Rs[j * 2 + 0] = (T)(l1 * o[0]);
  Rs[j * 2 + 1] = (T)(l2 * w1p2);
  Ss[j * 2 + 0] = s1;
  Ss[j * 2 + 1] = s2;
  ls[0][threadIdx.x] = (double)s1;
  ls[1][threadIdx.x] = (double)s2;
  __syncthreads();
  // S^T C: thread (g, c) = (tid / pp, tid % pp) sums rows g, g + G, ... of
  // the block (G = 256 / pp groups), then the groups are added in order
  const int64_t r0 = (int64_t)blockIdx.x * 256;
  const int G = 256 / pp;
  const int c = (int)threadIdx.x % pp, g = (int)threadIdx.x / pp;
  double a0 = 0.0, a1 = 0.0;
  for (int r = g; r < 256; r += G) {
    const double cv = (double)C[(r0 + r) * pp + c];
    a0 = fma(ls[0][r], cv, a0);
    a1 = fma(ls[1][r], cv, a1);
  }
  red[0][threadIdx.x] = a0;
  red[1][threadIdx.x] = a1;
  const double vj = (double)v[j];
  double* out = spart + (int64_t)blockIdx.x * (2 * pp + 2);
  __syncthreads();
  if ((int)threadIdx.x < 2 * pp) {
    const int e = (int)threadIdx.x / pp, cc = (int)threadIdx.x % pp;
    double acc = 0.0;
    for (int q = 0; q < G; ++q) acc += red[e][q * pp + cc];
    out[threadIdx.x] = acc;
  }
  __syncthreads();
  // S^T v
  red[0][threadIdx.x] = ls[0][threadIdx.x] * vj;
  red[1][threadIdx.x] = ls[1][threadIdx.x] * vj;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 2) out[2 * pp + threadIdx.x] = red[threadIdx.x][0];
}

// beta += R (S^T C + (S^T v) uY) + (W v) uY;  C += v uY  (C = X^T Y; S^T C
// from the old C; st = [S^T C (2 x pp), S^T v (2)]), one thread per (row,
// column).  With X non-null (a row change
// u = e_row) the thread of column 0 also applies X[row][j] += v[j].
template <typename T>
__global__ void __launch_bounds__(256)
k_ols_beta(const T* __restrict__ Rs, const double* __restrict__ vec, const double* __restrict__ st,
           const double* __restrict__ uy, const T* __restrict__ v, T* __restrict__ beta, T* __restrict__ C,
           int64_t n_pad, int pp, T* __restrict__ X, int64_t row) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n_pad * pp; e += (int64_t)gridDim.x * 256) {
    const int64_t j = e / pp;
    const int c = (int)(e % pp);
    const double y = uy[c];
    double d = vec[j * 5 + 2] * y;
    d = fma((double)Rs[j * 2 + 0], st[c] + st[2 * pp] * y, d);
    d = fma((double)Rs[j * 2 + 1], st[pp + c] + st[2 * pp + 1] * y, d);
    const double vj = (double)v[j];
    beta[e] = (T)((double)beta[e] + d);
    C[e] = (T)((double)C[e] + vj * y);
    if (X != nullptr && c == 0) X[row * n_pad + j] = (T)((double)X[row * n_pad + j] + vj);
  }
}

// X += u v^T over the m_pad x n_pad matrix.
template <typename T>
__global__ void __launch_bounds__(256)
k_rank1(T* __restrict__ X, int64_t m_pad, int64_t n_pad, const T* __restrict__ u, const T* __restrict__ v) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < m_pad * n_pad; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / n_pad, j = e % n_pad;
    X[e] = (T)((double)X[e] + (double)u[i] * (double)v[j]);
  }
}

// Row change (u = e_row, v = dx): stages v (zero beyond n), the operand
// slabs with X^T u = X[row] and u^T u = 1, and u^T Y = Y[row].
template <typename T>
__global__ void __launch_bounds__(256)
k_ols_stage_row(const T* __restrict__ dx, int64_t n, const T* __restrict__ X, const T* __restrict__ Y, int64_t row,
                int64_t n_pad, int pp, T* __restrict__ vbuf, T* __restrict__ Pk, T* __restrict__ Qk,
                double* __restrict__ uy) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < pp) uy[j] = (double)Y[row * pp + j];
  if (j >= n_pad) return;
  const T vt = j < n ? dx[j] : T(0);
  const double vj = (double)vt, x = (double)X[row * n_pad + j];
  vbuf[j] = vt;
  Pk[j * 4 + 0] = vt;
  Pk[j * 4 + 1] = (T)(x + vj);
  Pk[j * 4 + 2] = vt;
  Pk[j * 4 + 3] = T(0);
  Qk[j * 4 + 0] = (T)x;
  Qk[j * 4 + 1] = vt;
  Qk[j * 4 + 2] = T(0);
  Qk[j * 4 + 3] = T(0);
}

}  // namespace
}  // namespace lv

struct lv_ols {
  int64_t m, n, p, m_pad, n_pad;
  int pp, elem, nct, nrt;
  lv_mode mode;
  size_t X, Y, W, C, beta, ubuf, vbuf, Pk, Qk, Rs, Ss, partX, partY, vec;
  size_t pXu, pUu, pUy, dpart, spart, sums, red;
  size_t Z, Xk, Xn, Tk, C64, B64;
  size_t total;
  char* base;
  int iterations;
  double residual, cond;
  template <typename T> T* at(size_t off) const { return reinterpret_cast<T*>(base + off); }
  double* d(size_t off) const { return reinterpret_cast<double*>(base + off); }
};

namespace {

lv_status check_ols(int64_t m, int64_t n, int64_t p, lv_mode mode) {
  if (mode != LV_FP64 && mode != LV_FP32) return fail(LV_EINVAL, "OLS views take LV_FP64 or LV_FP32, got %d", (int)mode);
  if (n < 1 || n > kOlsMaxOrder) return fail(LV_EINVAL, "n = %lld outside [1, %lld]", (long long)n, (long long)kOlsMaxOrder);
  if (m < n || m > (int64_t)1 << 22) return fail(LV_EINVAL, "m = %lld outside [n, 2^22]", (long long)m);
  if (p < 1 || p > kOlsMaxCols) return fail(LV_EINVAL, "p = %lld outside [1, %d]", (long long)p, kOlsMaxCols);
  return LV_OK;
}

void layout_ols(lv_ols& o, int64_t m, int64_t n, int64_t p, lv_mode mode) {
  o.m = m; o.n = n; o.p = p; o.mode = mode;
  o.elem = mode == LV_FP64 ? 8 : 4;
  o.m_pad = round_up(m, kPadOrder);
  o.n_pad = round_up(n, kPadOrder);
  o.pp = (int)next_pow2(p);
  o.nct = (int)(o.n_pad / tile_cols_bytes(o.elem));
  o.nrt = (int)((o.n_pad + kTileRows - 1) / kTileRows);
  const size_t e = o.elem, np = o.n_pad, mp = o.m_pad, pp = o.pp;
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t at = off; off = align_up(off + bytes); return at; };
  o.X = take(mp * np * e);
  o.Y = take(mp * pp * e);
  o.W = take(np * np * e);
  o.C = take(np * pp * e);
  o.beta = take(np * pp * e);
  o.ubuf = take(mp * e);
  o.vbuf = take(np * e);
  o.Pk = take(np * 4 * e);
  o.Qk = take(np * 4 * e);
  o.Rs = take(np * 2 * e);
  o.Ss = take(np * 2 * e);
  o.partX = take((size_t)o.nct * np * 4 * e);
  o.partY = take((size_t)o.nrt * np * 4 * e);
  o.vec = take(np * 5 * sizeof(double));
  o.pXu = take((mp / kAtbRows) * np * sizeof(double));
  o.pUu = take((mp / kAtbRows) * sizeof(double));
  o.pUy = take((mp / kAtbRows) * pp * sizeof(double));
  o.dpart = take((np / kVecRows) * 4 * sizeof(double));
  o.sums = take((8 + 2 * kOlsMaxCols + 2) * sizeof(double));
  o.spart = take((np / 256) * (2 * pp + 2) * sizeof(double));
  o.red = take((kRedBlocks + 8) * sizeof(double));
  o.Z = take(np * np * sizeof(double));
  o.Xk = take(np * np * sizeof(double));
  o.Xn = take(np * np * sizeof(double));
  o.Tk = take(np * np * sizeof(double));
  o.C64 = take(np * pp * sizeof(double));
  o.B64 = take(np * pp * sizeof(double));
  o.total = off;
}

// Re-evaluation from the stored X and Y: Z = X^T X and C = X^T Y in double,
// W = Z^{-1} by Newton-Schulz (X_0 = I / ||Z||_inf, which puts the spectrum
// of Z X_0 in (0, 1] for symmetric positive definite Z; each step squares
// the residual I - Z X), beta = W C; each rounded once to the storage type.
// Iterates until the residual max|Z X - I| stops halving (at most 100
// steps); fails if it is still above 1e-6 (Z singular or too ill-conditioned
// for the storage precision).
template <typename T>
lv_status ols_build(lv_ols* o, hipStream_t s) {
  const int64_t np = o->n_pad, mp = o->m_pad;
  const dim3 gz((unsigned)(np / 32), (unsigned)(np / 32));
  hipLaunchKernelGGL((k_tn_gemm<T>), gz, dim3(256), 0, s, o->at<T>(o->X), np, o->at<T>(o->X), np, o->d(o->Z), np,
                     mp, (int)np, (int)np);
  const dim3 gc((unsigned)(np / 32), (unsigned)((o->pp + 31) / 32));
  hipLaunchKernelGGL((k_tn_gemm<T>), gc, dim3(256), 0, s, o->at<T>(o->X), np, o->at<T>(o->Y), (int64_t)o->pp,
                     o->d(o->C64), (int64_t)o->pp, mp, (int)np, o->pp);
  hipLaunchKernelGGL(k_pad_square, dim3(kRedBlocks), dim3(256), 0, s, o->d(o->Z), o->n, np, false);
  // ||Z||_inf of the padded Z (its padding is the identity) scales X_0; the
  // norm of the unpadded block goes into the condition number
  hipLaunchKernelGGL(k_rowabs_max, dim3(kRedBlocks), dim3(256), 0, s, o->d(o->Z), np, np, o->d(o->red));
  hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, s, o->d(o->red), kRedBlocks, o->d(o->red) + kRedBlocks + 3);
  hipLaunchKernelGGL(k_scaled_identity, dim3(kRedBlocks), dim3(256), 0, s, o->d(o->Xk), np, o->d(o->red) + kRedBlocks + 3);
  hipLaunchKernelGGL(k_rowabs_max, dim3(kRedBlocks), dim3(256), 0, s, o->d(o->Z), o->n, np, o->d(o->red));
  hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, s, o->d(o->red), kRedBlocks, o->d(o->red) + kRedBlocks);
  lv_status st = hip_check(hipGetLastError(), "OLS setup");
  double* x = o->d(o->Xk);
  double* xn = o->d(o->Xn);
  double prev = 1e300, res = 1e300;
  int it = 0;
  for (; it < 100 && st == LV_OK; ++it) {
    st = hip_check(launch_gemm<double>(o->d(o->Z), np, x, np, o->d(o->Tk), np, np, s), "Z X");
    if (st != LV_OK) break;
    hipLaunchKernelGGL(k_ns_step, dim3(kRedBlocks), dim3(256), 0, s, o->d(o->Tk), np, o->d(o->red));
    hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, s, o->d(o->red), kRedBlocks, o->d(o->red) + kRedBlocks + 1);
    st = hip_check(hipMemcpyAsync(&res, o->d(o->red) + kRedBlocks + 1, sizeof(double), hipMemcpyDeviceToHost, s),
                   "residual");
    if (st == LV_OK) st = hip_check(hipStreamSynchronize(s), "residual sync");
    if (st != LV_OK) break;
    if (!(res < 1e300)) { st = fail(LV_EINVAL, "Newton-Schulz diverged: X^T X is not positive definite"); break; }
    if (res <= 1e-15 || (res > 0.5 * prev && res < 1e-6)) break;   // at the rounding floor: keep this X
    st = hip_check(launch_gemm<double>(x, np, o->d(o->Tk), np, xn, np, np, s), "X (2I - Z X)");
    double* t = x; x = xn; xn = t;
    prev = res;
  }
  o->iterations = it;
  o->residual = res;
  if (st != LV_OK) return st;
  if (!(res < 1e-6)) return fail(LV_EINVAL, "X^T X is singular or too ill-conditioned (residual %.3g)", res);
  // infinity-norm condition number ||Z|| ||W||: rounding can leave an
  // exactly singular Z with tiny nonzero eigenvalues, which the iteration
  // then inverts; reject what the storage precision cannot represent
  hipLaunchKernelGGL(k_rowabs_max, dim3(kRedBlocks), dim3(256), 0, s, x, o->n, np, o->d(o->red));
  hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, s, o->d(o->red), kRedBlocks, o->d(o->red) + kRedBlocks + 2);
  double norms[3] = {0.0, 0.0, 0.0};
  st = hip_check(hipMemcpyAsync(norms, o->d(o->red) + kRedBlocks, 3 * sizeof(double), hipMemcpyDeviceToHost, s),
                 "norms");
  if (st == LV_OK) st = hip_check(hipStreamSynchronize(s), "norms sync");
  if (st != LV_OK) return st;
  o->cond = norms[0] * norms[2];
  const double unit = sizeof(T) == 8 ? 0x1p-53 : 0x1p-24;
  if (!(o->cond * unit < 0.1))
    return fail(LV_EINVAL, "X^T X is singular or too ill-conditioned (condition number %.3g)", o->cond);
  hipLaunchKernelGGL(k_pad_square, dim3(kRedBlocks), dim3(256), 0, s, x, o->n, np, true);
  st = hip_check(launch_copy_pad<double, T>(x, np, np, o->at<T>(o->W), np, np, s), "round W");
  if (st == LV_OK) st = hip_check(launch_gemm_np(o->pp, x, np, o->d(o->C64), o->d(o->B64), nullptr, np, s), "W C");
  if (st == LV_OK)
    st = hip_check(launch_copy_rect<double, T>(o->d(o->C64), o->pp, np, o->pp, o->at<T>(o->C), np, o->pp, s), "round C");
  if (st == LV_OK)
    st = hip_check(launch_copy_rect<double, T>(o->d(o->B64), o->pp, np, o->pp, o->at<T>(o->beta), np, o->pp, s),
                   "round beta");
  return st;
}

// One update.  row >= 0: the row change Delta X = e_row dx^T (dx: n values
// on the device, staged here); else Delta X = u v^T with u, v staged in
// ubuf, vbuf.  Launches: staging (row) or X^T u, u^T u, u^T Y and the
// operand slabs (dense); the read-only pass over W; vectors and dot
// partials; factors R, S and the S^T C, S^T v partials; W += R S^T; beta
// and C (and the row of X); X += u v^T (dense).
template <typename T>
lv_status ols_update(lv_ols* o, int64_t row, const T* dx, hipStream_t s) {
  const int64_t np = o->n_pad, mp = o->m_pad;
  const int pp = o->pp;
  const unsigned gv = (unsigned)(np / 256);
  lv_status st = LV_OK;
  if (row >= 0) {
    hipLaunchKernelGGL((k_ols_stage_row<T>), dim3(gv), dim3(256), 0, s, dx, o->n, o->at<T>(o->X), o->at<T>(o->Y), row,
                       np, pp, o->at<T>(o->vbuf), o->at<T>(o->Pk), o->at<T>(o->Qk), o->d(o->pUy));
    st = hip_check(hipGetLastError(), "row stage");
  } else {
    st = hip_check(launch_atb<T>(1, (int)np, o->at<T>(o->ubuf), 1, o->at<T>(o->X), np, mp, o->d(o->pXu), s), "X^T u");
    if (st == LV_OK) st = hip_check(launch_atb<T>(1, 1, o->at<T>(o->ubuf), 1, o->at<T>(o->ubuf), 1, mp, o->d(o->pUu), s), "u^T u");
    if (st == LV_OK)
      st = hip_check(launch_atb<T>(1, pp, o->at<T>(o->ubuf), 1, o->at<T>(o->Y), pp, mp, o->d(o->pUy), s), "u^T Y");
    if (st == LV_OK) {
      hipLaunchKernelGGL((k_ols_operands<T>), dim3(gv), dim3(256), 0, s, o->d(o->pXu), o->d(o->pUu),
                         o->at<T>(o->vbuf), o->at<T>(o->Pk), o->at<T>(o->Qk), np);
      st = hip_check(hipGetLastError(), "operands");
    }
  }
  if (st == LV_OK)
    st = hip_check(launch_level_readonly<T>(4, o->at<T>(o->W), np, np, kTileRows, o->at<T>(o->Pk), o->at<T>(o->Qk), 4,
                                            o->at<T>(o->partX), o->at<T>(o->partY), s),
                   "W [p1 p2 v], W^T [q1 q2]");
  if (st != LV_OK) return st;
  const int nvb = (int)(np / kVecRows);
  hipLaunchKernelGGL((k_ols_vectors<T>), dim3((unsigned)nvb), dim3(256), 0, s, o->at<T>(o->partX), o->nct,
                     o->at<T>(o->partY), o->nrt, np, o->at<T>(o->Pk), o->at<T>(o->Qk), o->d(o->vec), o->d(o->dpart));
  hipLaunchKernelGGL(k_sum_partials, dim3(4), dim3(256), 0, s, o->d(o->dpart), nvb, 4, o->d(o->sums));
  hipLaunchKernelGGL((k_ols_rs<T>), dim3(gv), dim3(256), 0, s, o->d(o->vec), o->d(o->sums),
                     o->at<T>(o->Rs), o->at<T>(o->Ss), o->at<T>(o->C), o->at<T>(o->vbuf), pp, o->d(o->spart));
  st = hip_check(hipGetLastError(), "Sherman-Morrison factors");
  if (st == LV_OK)
    st = hip_check(launch_level_update<T>(2, o->at<T>(o->W), np, np, o->at<T>(o->Rs), o->at<T>(o->Ss), 2, s),
                   "W += R S^T");
  if (st != LV_OK) return st;
  hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)(2 * pp + 2)), dim3(256), 0, s, o->d(o->spart), (int)gv,
                     2 * pp + 2, o->d(o->sums) + 8);
  hipLaunchKernelGGL((k_ols_beta<T>), dim3((unsigned)((np * pp + 255) / 256)), dim3(256), 0, s, o->at<T>(o->Rs),
                     o->d(o->vec), o->d(o->sums) + 8, o->d(o->pUy), o->at<T>(o->vbuf), o->at<T>(o->beta),
                     o->at<T>(o->C), np, pp, row >= 0 ? o->at<T>(o->X) : nullptr, row);
  if (row < 0)
    hipLaunchKernelGGL((k_rank1<T>), dim3(2048), dim3(256), 0, s, o->at<T>(o->X), mp, np, o->at<T>(o->ubuf),
                       o->at<T>(o->vbuf));
  return hip_check(hipGetLastError(), "beta, X");
}

}  // namespace

extern "C" {

size_t lv_ols_footprint(int64_t m, int64_t n, int64_t p, lv_mode mode) {
  if (check_ols(m, n, p, mode) != LV_OK) return 0;
  lv_ols o;
  layout_ols(o, m, n, p, mode);
  return o.total;
}

lv_status lv_ols_create(const void* X, int64_t m, int64_t n, int64_t ldx, const void* Y, int64_t p, int64_t ldy,
                        lv_mode mode, void* workspace, size_t ws_bytes, void* stream, lv_ols** out) {
  g_err[0] = 0;
  if (!out) return fail(LV_EINVAL, "out is NULL");
  *out = nullptr;
  lv_status st = check_ols(m, n, p, mode);
  if (st != LV_OK) return st;
  if (!X || !Y || !workspace) return fail(LV_EINVAL, "X, Y or workspace is NULL");
  if (ldx < n || ldy < p) return fail(LV_EINVAL, "ldx < n or ldy < p");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(LV_ENOMEM, "workspace is not %zu-byte aligned", kAlign);
  lv_ols* o = new (std::nothrow) lv_ols();
  if (!o) return fail(LV_ENOMEM, "host allocation of the OLS handle failed");
  layout_ols(*o, m, n, p, mode);
  if (ws_bytes < o->total) {
    const size_t need = o->total;
    delete o;
    return fail(LV_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  }
  o->base = static_cast<char*>(workspace);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (mode == LV_FP64) {
    st = hip_check(launch_copy_rect<double, double>(static_cast<const double*>(X), ldx, m, (int)n, o->at<double>(o->X),
                                                    o->m_pad, (int)o->n_pad, s), "copy X");
    if (st == LV_OK)
      st = hip_check(launch_copy_rect<double, double>(static_cast<const double*>(Y), ldy, m, (int)p,
                                                      o->at<double>(o->Y), o->m_pad, o->pp, s), "copy Y");
    if (st == LV_OK) st = ols_build<double>(o, s);
  } else {
    st = hip_check(launch_copy_rect<float, float>(static_cast<const float*>(X), ldx, m, (int)n, o->at<float>(o->X),
                                                  o->m_pad, (int)o->n_pad, s), "copy X");
    if (st == LV_OK)
      st = hip_check(launch_copy_rect<float, float>(static_cast<const float*>(Y), ldy, m, (int)p, o->at<float>(o->Y),
                                                    o->m_pad, o->pp, s), "copy Y");
    if (st == LV_OK) st = ols_build<float>(o, s);
  }
  if (st != LV_OK) { delete o; return st; }
  *out = o;
  return LV_OK;
}

lv_status lv_ols_update(lv_ols* o, const void* u, const void* v, void* stream) {
  g_err[0] = 0;
  if (!o || !u || !v) return fail(LV_EINVAL, "handle, u or v is NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  lv_status st;
  if (o->mode == LV_FP64) {
    st = hip_check(launch_copy_rect<double, double>(static_cast<const double*>(u), 1, o->m, 1, o->at<double>(o->ubuf),
                                                    o->m_pad, 1, s), "stage u");
    if (st == LV_OK)
      st = hip_check(launch_copy_rect<double, double>(static_cast<const double*>(v), 1, o->n, 1,
                                                      o->at<double>(o->vbuf), o->n_pad, 1, s), "stage v");
    return st == LV_OK ? ols_update<double>(o, -1, nullptr, s) : st;
  }
  st = hip_check(launch_copy_rect<float, float>(static_cast<const float*>(u), 1, o->m, 1, o->at<float>(o->ubuf),
                                                o->m_pad, 1, s), "stage u");
  if (st == LV_OK)
    st = hip_check(launch_copy_rect<float, float>(static_cast<const float*>(v), 1, o->n, 1, o->at<float>(o->vbuf),
                                                  o->n_pad, 1, s), "stage v");
  return st == LV_OK ? ols_update<float>(o, -1, nullptr, s) : st;
}

lv_status lv_ols_update_row(lv_ols* o, int64_t row, const void* dx, void* stream) {
  g_err[0] = 0;
  if (!o || !dx) return fail(LV_EINVAL, "handle or dx is NULL");
  if (row < 0 || row >= o->m) return fail(LV_EINVAL, "row %lld outside [0, %lld)", (long long)row, (long long)o->m);
  hipStream_t s = static_cast<hipStream_t>(stream);
  return o->mode == LV_FP64 ? ols_update<double>(o, row, static_cast<const double*>(dx), s)
                            : ols_update<float>(o, row, static_cast<const float*>(dx), s);
}

lv_status lv_ols_read(const lv_ols* o, int what, void* out, int64_t ldo, void* stream) {
  g_err[0] = 0;
  if (!o || !out) return fail(LV_EINVAL, "handle or out is NULL");
  const size_t es = o->elem;
  size_t off;
  int64_t rows, cols, ld;
  switch (what) {
    case LV_OLS_BETA: off = o->beta; rows = o->n; cols = o->p; ld = o->pp; break;
    case LV_OLS_INVERSE: off = o->W; rows = o->n; cols = o->n; ld = o->n_pad; break;
    case LV_OLS_X: off = o->X; rows = o->m; cols = o->n; ld = o->n_pad; break;
    default: return fail(LV_EINVAL, "unknown OLS quantity %d", what);
  }
  if (ldo < cols) return fail(LV_EINVAL, "ldo < %lld", (long long)cols);
  return hip_check(hipMemcpy2DAsync(out, ldo * es, o->base + off, ld * es, cols * es, rows, hipMemcpyDeviceToDevice,
                                    static_cast<hipStream_t>(stream)),
                   "read");
}

lv_status lv_ols_info(const lv_ols* o, int* iterations, double* residual, double* cond) {
  if (!o) return fail(LV_EINVAL, "handle is NULL");
  if (iterations) *iterations = o->iterations;
  if (residual) *residual = o->residual;
  if (cond) *cond = o->cond;
  return LV_OK;
}

void lv_ols_destroy(lv_ols* o) { delete o; }

}  // extern "C"
