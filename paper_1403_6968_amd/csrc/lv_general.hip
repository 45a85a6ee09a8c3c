// General iterative form T_{i+1} = A T_i + B (LINVIEW Sec. 5.3, Table 1,
// exponential model: T_1 = A T_0 + B, T_{2i} = P_i T_i + S_i B), maintained
// by hybrid evaluation: the change of every stored T_i is one dense n x p
// matrix D_i (Sec. 5.3.2, "Hybrid evaluation"), obtained from the old values
// by the delta rule of Sec. 4.1:
//     D_1 = U (V^T T_0),
//     D_{2i} = P_i D_i + U_i (V_i^T (T_i + D_i)) + Q_i (W_i^T B)
// with Delta P_i = U_i V_i^T, Delta S_i = Q_i W_i^T.  The products P_i D_i
// run as read-only skinny passes (lv_fused.hip / lv_skinny.hip); this file
// holds the small reductions A^T B, the tail that assembles D_{2i} and adds
// it to T_{2i}, and the (n x n)(n x p) product used at creation; and, for
// incremental evaluation with factored deltas Delta T_i = Y_i Z_i^T (App. B),
//     Y_{2i} = [U_i, P_i Y_i + U_i (V_i^T Y_i), Q_i],  Z_{2i} = [T_i^T V_i, Z_i, B^T W_i],
// the kernels that assemble the new factor slabs (Z kept transposed, factor-
// major) and apply T_i += Y_i Z_i^T.
#include "lv_device.h"
#include "lv_view_impl.h"

namespace lv {
namespace {

// part[tile][a * p + b] = sum over the tile's rows of A[row][a] B[row][b]
// (double), pairs (a, b) spread over threads and blocks.
template <typename T>
__global__ void __launch_bounds__(256)
k_atb(const T* __restrict__ A, int64_t lda, const T* __restrict__ B, int64_t ldb, int R, int p,
      double* __restrict__ part) {
  const int tile = blockIdx.x;
  const int pair = blockIdx.y * 256 + threadIdx.x;
  if (pair >= R * p) return;
  const int a = pair / p, b = pair % p;
  const int64_t r0 = (int64_t)tile * kAtbRows;
  double acc = 0.0;
#pragma unroll 8
  for (int i = 0; i < kAtbRows; ++i) acc = fma((double)A[(r0 + i) * lda + a], (double)B[(r0 + i) * ldb + b], acc);
  part[(int64_t)tile * R * p + pair] = acc;
}

// One thread per (row, column) of the n_pad x pp delta:
//   d = sum_t partX[t][row][col] (t ascending, double)
//     + sum_c U[row][c] a[c][col] + sum_c Q[row][c] b[c][col]  (Q, b optional)
//   D[row][col] = d;  T[row][col] += d.
template <typename T>
__global__ void __launch_bounds__(256)
k_general_tail(const T* __restrict__ partX, int nct, const T* __restrict__ U, const T* __restrict__ Q, int W, int R,
               const double* __restrict__ a, const double* __restrict__ b, T* __restrict__ D, T* __restrict__ Tm,
               int64_t n_pad, int pp) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n_pad * pp) return;
  const int64_t row = idx / pp;
  const int col = (int)(idx % pp);
  double d = 0.0;
  const int64_t stride = n_pad * pp;
  for (int t = 0; t < nct; ++t) d += (double)partX[t * stride + idx];
  for (int c = 0; c < R; ++c) d = fma((double)U[row * W + c], a[c * pp + col], d);
  if (Q != nullptr)
    for (int c = 0; c < R; ++c) d = fma((double)Q[row * W + c], b[c * pp + col], d);
  D[idx] = (T)d;
  Tm[idx] = (T)((double)Tm[idx] + d);
}

// C = A B (+ C0) for A n_pad x n_pad (lda), B n_pad x PP (ld PP), double:
// one wave per row, lanes split the summation index, xor-shuffle reduction.
template <int PP>
__global__ void __launch_bounds__(256)
k_gemm_np(const double* __restrict__ A, int64_t lda, const double* __restrict__ B, double* __restrict__ C,
          const double* __restrict__ C0, int64_t n_pad, const int* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  double acc[PP];
#pragma unroll
  for (int c = 0; c < PP; ++c) acc[c] = 0.0;
  for (int64_t k = lane; k < n_pad; k += 64) {
    const double x = A[row * lda + k];
#pragma unroll
    for (int c = 0; c < PP; ++c) acc[c] = fma(x, B[k * PP + c], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < PP; ++c) {
    double v = acc[c];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    acc[c] = v;
  }
  if (lane < PP) {
    double out = 0.0;
#pragma unroll
    for (int c = 0; c < PP; ++c) out = lane == c ? acc[c] : out;
    C[row * PP + lane] = out + (C0 != nullptr ? C0[row * PP + lane] : 0.0);
  }
}

template <typename Tin, typename Tout>
__global__ void __launch_bounds__(256)
k_copy_rect(const Tin* __restrict__ src, int64_t lds, int64_t n, int p, Tout* __restrict__ dst, int64_t n_pad, int pp,
            const int* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n_pad * pp) return;
  const int64_t row = idx / pp;
  const int col = (int)(idx % pp);
  dst[idx] = (row < n && col < p) ? (Tout)src[row * lds + col] : Tout(0);
}

// Factored deltas: one thread per (row, column) of the new Y slab.
template <typename T>
__global__ void __launch_bounds__(256)
k_gfac_y(const T* __restrict__ partX, int nct, int pR, const T* __restrict__ U, const T* __restrict__ Q, int W, int R,
         const double* __restrict__ G, int ldg, int wy, T* __restrict__ Ynew, int WYn, int64_t n_pad) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n_pad * WYn) return;
  const int64_t row = idx / WYn;
  const int col = (int)(idx % WYn);
  double y = 0.0;
  if (col < R) {
    y = (double)U[row * W + col];
  } else if (col < R + wy) {
    const int c = col - R;
    for (int t = 0; t < nct; ++t) y += (double)partX[((int64_t)t * n_pad + row) * pR + c];
    for (int d = 0; d < R; ++d) y = fma((double)U[row * W + d], G[d * ldg + c], y);
  } else if (col < 2 * R + wy && Q != nullptr) {
    y = (double)Q[row * W + (col - R - wy)];
  }
  Ynew[idx] = (T)y;
}

// One thread per (factor row, column of T) of the new Zt slab.
template <typename T>
__global__ void __launch_bounds__(256)
k_gfac_z(const double* __restrict__ a, const T* __restrict__ Zt, int wy, const double* __restrict__ b, int R,
         T* __restrict__ Ztnew, int WYn, int pp) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)WYn * pp) return;
  const int crow = (int)(idx / pp);
  const int col = (int)(idx % pp);
  T z = T(0);
  if (crow < R) z = (T)a[(int64_t)crow * pp + col];
  else if (crow < R + wy) z = Zt[(int64_t)(crow - R) * pp + col];
  else if (crow < 2 * R + wy && b != nullptr) z = (T)b[(int64_t)(crow - R - wy) * pp + col];
  Ztnew[idx] = z;
}

// Tm[row][col] += sum_c Y[row][c] Zt[c][col] (double), one thread per element.
template <typename T>
__global__ void __launch_bounds__(256)
k_rank_rect(T* __restrict__ Tm, const T* __restrict__ Y, int sy, const T* __restrict__ Zt, int w, int64_t n_pad,
            int pp) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n_pad * pp) return;
  const int64_t row = idx / pp;
  const int col = (int)(idx % pp);
  double d = 0.0;
  for (int c = 0; c < w; ++c) d = fma((double)Y[row * sy + c], (double)Zt[(int64_t)c * pp + col], d);
  Tm[idx] = (T)((double)Tm[idx] + d);
}

// The same for a 4 x 4 block per thread (four rows, four consecutive
// columns; n_pad and pp multiples of 4): each Zt row segment is loaded once
// for the four rows, each Y value once for the four columns.
template <typename T>
__global__ void __launch_bounds__(256)
k_rank_rect4(T* __restrict__ Tm, const T* __restrict__ Y, int sy, const T* __restrict__ Zt, int w, int64_t n_pad,
             int pp) {
  typedef T v4 __attribute__((ext_vector_type(4)));
  const int q4 = pp / 4;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (n_pad / 4) * q4) return;
  const int64_t row0 = (idx / q4) * 4;
  const int col = (int)(idx % q4) * 4;
  double d[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) d[a][b] = 0.0;
  for (int c = 0; c < w; ++c) {
    const v4 z = *reinterpret_cast<const v4*>(Zt + (int64_t)c * pp + col);
    const double zz[4] = {(double)z.x, (double)z.y, (double)z.z, (double)z.w};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const double y = (double)Y[(row0 + a) * sy + c];
#pragma unroll
      for (int b = 0; b < 4; ++b) d[a][b] = fma(y, zz[b], d[a][b]);
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    v4* tp = reinterpret_cast<v4*>(Tm + (row0 + a) * pp + col);
    v4 t = *tp;
    t.x = (T)((double)t.x + d[a][0]);
    t.y = (T)((double)t.y + d[a][1]);
    t.z = (T)((double)t.z + d[a][2]);
    t.w = (T)((double)t.w + d[a][3]);
    *tp = t;
  }
}

}  // namespace

template <typename T>
hipError_t launch_gfac_y(const T* partX, int nct, int pR, const T* U, const T* Q, int W, int R, const double* G,
                         int ldg, int wy, T* Ynew, int WYn, int64_t n_pad, hipStream_t s) {
  hipLaunchKernelGGL((k_gfac_y<T>), dim3((unsigned)((n_pad * WYn + 255) / 256)), dim3(256), 0, s, partX, nct, pR, U, Q,
                     W, R, G, ldg, wy, Ynew, WYn, n_pad);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gfac_z(const double* a, const T* Zt, int wy, const double* b, int R, T* Ztnew, int WYn, int pp,
                         hipStream_t s) {
  hipLaunchKernelGGL((k_gfac_z<T>), dim3((unsigned)(((int64_t)WYn * pp + 255) / 256)), dim3(256), 0, s, a, Zt, wy, b,
                     R, Ztnew, WYn, pp);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rank_rect(T* Tm, const T* Y, int sy, const T* Zt, int w, int64_t n_pad, int pp, hipStream_t s) {
  if (pp % 4 == 0 && n_pad % 4 == 0) {
    hipLaunchKernelGGL((k_rank_rect4<T>), dim3((unsigned)((n_pad / 4 * (pp / 4) + 255) / 256)), dim3(256), 0, s, Tm,
                       Y, sy, Zt, w, n_pad, pp);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_rank_rect<T>), dim3((unsigned)((n_pad * pp + 255) / 256)), dim3(256), 0, s, Tm, Y, sy, Zt, w,
                     n_pad, pp);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_atb(int R, int p, const T* A, int64_t lda, const T* B, int64_t ldb, int64_t n_pad, double* part,
                      hipStream_t s) {
  const int ntile = (int)(n_pad / kAtbRows);
  const dim3 grid((unsigned)ntile, (unsigned)((R * p + 255) / 256));
  hipLaunchKernelGGL((k_atb<T>), grid, dim3(256), 0, s, A, lda, B, ldb, R, p, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_gram_sum(part, ntile, R * p, s);
}

template <typename T>
hipError_t launch_general_tail(const T* partX, int nct, const T* U, const T* Q, int W, int R, const double* a,
                               const double* b, T* D, T* Tm, int64_t n_pad, int pp, hipStream_t s) {
  hipLaunchKernelGGL((k_general_tail<T>), dim3((unsigned)((n_pad * pp + 255) / 256)), dim3(256), 0, s, partX, nct, U,
                     Q, W, R, a, b, D, Tm, n_pad, pp);
  return hipGetLastError();
}

hipError_t launch_gemm_np(int pp, const double* A, int64_t lda, const double* B, double* C, const double* C0,
                          int64_t n_pad, hipStream_t s, const int* gate) {
  const dim3 grid((unsigned)(n_pad / 4));
  switch (pp) {
#define LV_CASE(PPV) case PPV: hipLaunchKernelGGL((k_gemm_np<PPV>), grid, dim3(256), 0, s, A, lda, B, C, C0, n_pad, gate); break;
    LV_CASE(1) LV_CASE(2) LV_CASE(4) LV_CASE(8) LV_CASE(16) LV_CASE(32) LV_CASE(64)
#undef LV_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename Tin, typename Tout>
hipError_t launch_copy_rect(const Tin* src, int64_t lds, int64_t n, int p, Tout* dst, int64_t n_pad, int pp,
                            hipStream_t s, const int* gate) {
  hipLaunchKernelGGL((k_copy_rect<Tin, Tout>), dim3((unsigned)((n_pad * pp + 255) / 256)), dim3(256), 0, s, src, lds,
                     n, p, dst, n_pad, pp, gate);
  return hipGetLastError();
}

#define LV_INST(T)                                                                                            \
  template hipError_t launch_atb<T>(int, int, const T*, int64_t, const T*, int64_t, int64_t, double*,         \
                                    hipStream_t);                                                             \
  template hipError_t launch_general_tail<T>(const T*, int, const T*, const T*, int, int, const double*,       \
                                             const double*, T*, T*, int64_t, int, hipStream_t);
LV_INST(float)
LV_INST(double)
#undef LV_INST
#define LV_INST(T)                                                                                             \
  template hipError_t launch_gfac_y<T>(const T*, int, int, const T*, const T*, int, int, const double*, int, int, \
                                       T*, int, int64_t, hipStream_t);                                         \
  template hipError_t launch_gfac_z<T>(const double*, const T*, int, const double*, int, T*, int, int,         \
                                       hipStream_t);                                                           \
  template hipError_t launch_rank_rect<T>(T*, const T*, int, const T*, int, int64_t, int, hipStream_t);
LV_INST(float)
LV_INST(double)
#undef LV_INST
template hipError_t launch_copy_rect<float, float>(const float*, int64_t, int64_t, int, float*, int64_t, int,
                                                   hipStream_t, const int*);
template hipError_t launch_copy_rect<double, double>(const double*, int64_t, int64_t, int, double*, int64_t, int,
                                                     hipStream_t, const int*);
template hipError_t launch_copy_rect<float, double>(const float*, int64_t, int64_t, int, double*, int64_t, int,
                                                    hipStream_t, const int*);
template hipError_t launch_copy_rect<double, float>(const double*, int64_t, int64_t, int, float*, int64_t, int,
                                                    hipStream_t, const int*);

}  // namespace lv
