// Dense MFMA products for view creation / re-anchoring (double) and for the
// re-evaluation baseline (double or float): C = A * B, n_pad x n_pad,
// row-major, n_pad a multiple of 256 (the repeated squarings of Table 1's
// exponential model, P_i = P_{i/2} P_{i/2}); launch_gemm_rect runs the same
// kernel on an M x K by K x N product (M, N multiples of 128, K of 16).
//
// Block tile 128 x 128 x 16, 256 threads as a 2 x 2 grid of waves, each wave
// owning a 64 x 64 sub-tile of C built from MFMA blocks:
//   double: v_mfma_f64_16x16x4f64 (4 x 4 blocks of 16 x 16)
//   float : v_mfma_f32_32x32x2f32 (2 x 2 blocks of 32 x 32)
// A and B tiles are staged through double-buffered LDS (A stored k-major so
// that the MFMA operand of a lane is one LDS element); the next K tile is
// fetched into registers while the current one feeds the matrix cores.
#include "lv_internal.h"

namespace lv {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

template <typename T> struct Mfma;

// A operand: lane supplies A[m = lane % 16][k = lane / 16];
// B operand: lane supplies B[k = lane / 16][n = lane % 16];
// result element v of a lane is C[lane / 16 + 4 * v][lane % 16].
template <> struct Mfma<double> {
  static constexpr int M = 16, K = 4, NACC = 4;
  using acc_t = v4d;
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int crow(int lane, int v) { return lane / 16 + 4 * v; }
};

// A operand: lane supplies A[m = lane % 32][k = lane / 32];
// B operand: lane supplies B[k = lane / 32][n = lane % 32];
// result element v of a lane is C[8 * (v / 4) + 4 * (lane / 32) + v % 4][lane % 32].
template <> struct Mfma<float> {
  static constexpr int M = 32, K = 2, NACC = 16;
  using acc_t = v16f;
  __device__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
  __device__ static int crow(int lane, int v) { return 8 * (v / 4) + 4 * (lane / 32) + (v % 4); }
};

constexpr int BM = 128, BN = 128, BK = 16;

template <typename T>
__global__ void __launch_bounds__(256)
k_gemm(const T* __restrict__ A, int64_t lda, const T* __restrict__ B, int64_t ldb,
       T* __restrict__ C, int64_t ldc, int n_pad, const int* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  using F = Mfma<T>;
  constexpr int M = F::M;
  constexpr int NB = 64 / M;           // MFMA blocks per wave per dimension
  constexpr int PADA = 4, PADB = 4;
  __shared__ T As[2][BK][BM + PADA];
  __shared__ T Bs[2][BK][BN + PADB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * BM;
  const int n0 = blockIdx.x * BN;

  // Global fetch assignment: 8 elements of A (row ar, k ak..ak+7) and of B
  // (row bk, columns bc..bc+7) per thread.
  const int ar = tid >> 1, ak = (tid & 1) * 8;
  const int bk = tid >> 4, bc = (tid & 15) * 8;
  T ra[8], rb[8];

  auto fetch = [&](int k0) {
    const T* pa = A + (int64_t)(m0 + ar) * lda + k0 + ak;
    const T* pb = B + (int64_t)(k0 + bk) * ldb + n0 + bc;
#pragma unroll
    for (int e = 0; e < 8; ++e) { ra[e] = pa[e]; rb[e] = pb[e]; }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 8; ++e) { As[buf][ak + e][ar] = ra[e]; Bs[buf][bk][bc + e] = rb[e]; }
  };

  typename F::acc_t acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int v = 0; v < F::NACC; ++v) acc[i][j][v] = T(0);

  const int nk = n_pad / BK;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) fetch((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += F::K) {
      T a[NB], b[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) a[i] = As[cur][ks + lane / M][wm * 64 + i * M + lane % M];
#pragma unroll
      for (int j = 0; j < NB; ++j) b[j] = Bs[cur][ks + lane / M][wn * 64 + j * M + lane % M];
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = F::mma(a[i], b[j], acc[i][j]);
    }
    if (kt + 1 < nk) stash(cur ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int v = 0; v < F::NACC; ++v) {
        const int r = m0 + wm * 64 + i * M + F::crow(lane, v);
        const int c = n0 + wn * 64 + j * M + lane % M;
        C[(int64_t)r * ldc + c] = acc[i][j][v];
      }
}

}  // namespace

template <typename T>
hipError_t launch_gemm(const T* A, int64_t lda, const T* B, int64_t ldb, T* C, int64_t ldc,
                       int64_t n_pad, hipStream_t s, const int* gate) {
  if (n_pad % BM != 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(n_pad / BN), (unsigned)(n_pad / BM));
  hipLaunchKernelGGL((k_gemm<T>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, (int)n_pad, gate);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gemm_rect(const T* A, int64_t lda, const T* B, int64_t ldb, T* C, int64_t ldc, int64_t M,
                            int64_t N, int64_t K, hipStream_t s, const int* gate) {
  if (M % BM != 0 || N % BN != 0 || K % BK != 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(N / BN), (unsigned)(M / BM));
  hipLaunchKernelGGL((k_gemm<T>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, (int)K, gate);
  return hipGetLastError();
}

template hipError_t launch_gemm_rect<double>(const double*, int64_t, const double*, int64_t, double*, int64_t,
                                             int64_t, int64_t, int64_t, hipStream_t, const int*);
template hipError_t launch_gemm_rect<float>(const float*, int64_t, const float*, int64_t, float*, int64_t,
                                            int64_t, int64_t, int64_t, hipStream_t, const int*);
template hipError_t launch_gemm<double>(const double*, int64_t, const double*, int64_t, double*,
                                        int64_t, int64_t, hipStream_t, const int*);
template hipError_t launch_gemm<float>(const float*, int64_t, const float*, int64_t, float*,
                                       int64_t, int64_t, hipStream_t, const int*);

}  // namespace lv
