// Drift check of a view's stored chain.  The exponential model defines every
// stored power by P_{2i} = P_i P_i (Table 1); incremental updates keep that
// relation only up to accumulated rounding.  A randomized (Freivalds-style)
// test measures, for a vector z and every level j,
//     rho_j = max|P_{j+1} z - P_j (P_j z)| / max|P_{j+1} z|
// with double accumulation over the stored values; when some rho_j exceeds
// the bound, the squaring chain is recomputed from the stored A by kernels
// that read the device-side gate written here (no host round trip).
#include "lv_internal.h"

namespace lv {
namespace {

template <typename T> struct alignas(16) V16 { T v[16 / sizeof(T)]; };

__global__ void __launch_bounds__(256)
k_vec_pad(const double* __restrict__ z, int64_t n, double* __restrict__ x, int64_t n_pad) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n_pad) x[i] = i < n ? z[i] : 0.0;
}

// y = P x: each wave owns 8 consecutive rows; lanes stride the columns in
// 16-byte vectors; the x values a lane needs are reused across the 8 rows.
template <typename T>
__global__ void __launch_bounds__(256)
k_matvec(const T* __restrict__ P, int64_t ldp, int n_pad, const double* __restrict__ x,
         double* __restrict__ y) {
  constexpr int EPL = 16 / (int)sizeof(T);
  constexpr int RW = 8;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + wave) * RW;
  if (r0 >= n_pad) return;
  double acc[RW];
#pragma unroll
  for (int t = 0; t < RW; ++t) acc[t] = 0.0;
  for (int c = lane * EPL; c < n_pad; c += 64 * EPL) {
    double xv[EPL];
#pragma unroll
    for (int e = 0; e < EPL; ++e) xv[e] = x[c + e];
#pragma unroll
    for (int t = 0; t < RW; ++t) {
      const V16<T> p = *reinterpret_cast<const V16<T>*>(P + (r0 + t) * ldp + c);
#pragma unroll
      for (int e = 0; e < EPL; ++e) acc[t] = fma((double)p.v[e], xv[e], acc[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < RW; ++t) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc[t] += __shfl_xor(acc[t], off);
  }
  if (lane == 0) {
#pragma unroll
    for (int t = 0; t < RW; ++t) y[r0 + t] = acc[t];
  }
}

// One block: maxima over all levels (order-independent), then the gate.
__global__ void __launch_bounds__(256)
k_drift_residual(const double* __restrict__ Pz, const double* __restrict__ PPz, int m,
                 int64_t n_pad, double tau, double* __restrict__ residuals, int* __restrict__ gate,
                 unsigned long long* __restrict__ counter) {
  __shared__ double sd[256], sc[256];
  __shared__ int fail;
  const int tid = threadIdx.x;
  if (tid == 0) fail = 0;
  for (int j = 0; j < m; ++j) {
    const double* c = Pz + (int64_t)(j + 1) * n_pad;
    const double* b = PPz + (int64_t)j * n_pad;
    double md = 0.0, mc = 0.0;
    for (int64_t i = tid; i < n_pad; i += 256) {
      md = fmax(md, fabs(c[i] - b[i]));
      mc = fmax(mc, fabs(c[i]));
    }
    sd[tid] = md;
    sc[tid] = mc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) {
        sd[tid] = fmax(sd[tid], sd[tid + w]);
        sc[tid] = fmax(sc[tid], sc[tid + w]);
      }
      __syncthreads();
    }
    if (tid == 0) {
      const double rho = sc[0] > 0.0 ? sd[0] / sc[0] : (sd[0] > 0.0 ? INFINITY : 0.0);
      residuals[j] = rho;
      if (!(rho <= tau)) fail = 1;  // also trips on NaN
    }
    __syncthreads();
  }
  if (tid == 0) {
    *gate = fail;
    if (fail) *counter += 1ull;
  }
}

// Probe vector of the periodic check when the caller gives none: entries
// +1 or -1 from the top bit of splitmix64 (Steele, Lea and Flood, 2014) of
// seed + i, zero beyond n.
__global__ void __launch_bounds__(256)
k_sign_vector(double* __restrict__ z, int64_t n, int64_t n_pad, unsigned long long seed) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n_pad) return;
  unsigned long long x = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(i + 1);
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  z[i] = i < n ? ((x >> 63) ? 1.0 : -1.0) : 0.0;
}

}  // namespace

hipError_t launch_sign_vector(double* z, int64_t n, int64_t n_pad, unsigned long long seed, hipStream_t s) {
  hipLaunchKernelGGL(k_sign_vector, dim3((unsigned)((n_pad + 255) / 256)), dim3(256), 0, s, z, n, n_pad, seed);
  return hipGetLastError();
}

hipError_t launch_vec_pad(const double* z, int64_t n, double* x, int64_t n_pad, hipStream_t s) {
  hipLaunchKernelGGL(k_vec_pad, dim3((unsigned)((n_pad + 255) / 256)), dim3(256), 0, s, z, n, x, n_pad);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_matvec(const T* P, int64_t ldp, int64_t n_pad, const double* x, double* y,
                         hipStream_t s) {
  const int64_t rows_per_block = 4 * 8;
  hipLaunchKernelGGL((k_matvec<T>), dim3((unsigned)((n_pad + rows_per_block - 1) / rows_per_block)),
                     dim3(256), 0, s, P, ldp, (int)n_pad, x, y);
  return hipGetLastError();
}

hipError_t launch_drift_residual(const double* Pz, const double* PPz, int m, int64_t n_pad,
                                 double tau, double* residuals, int* gate,
                                 unsigned long long* counter, hipStream_t s) {
  hipLaunchKernelGGL(k_drift_residual, dim3(1), dim3(256), 0, s, Pz, PPz, m, n_pad, tau, residuals,
                     gate, counter);
  return hipGetLastError();
}

template hipError_t launch_matvec<float>(const float*, int64_t, int64_t, const double*, double*,
                                         hipStream_t);
template hipError_t launch_matvec<double>(const double*, int64_t, int64_t, const double*, double*,
                                          hipStream_t);

}  // namespace lv
