// Generators of the stage-2 Toeplitz systems on the GPU (Sec. V): for each of
// B Hermitian positive definite Toeplitz matrices A_b (first column col_b,
// complex128) the first column x_b = A_b^{-1} e_0 by the Levinson recursion in
// float64, one workgroup per system.
//
// The monic vector a_k (A restricted to its leading k + 1 rows and columns
// maps a_k to err_k e_0, a_k[0] = 1) lives in LDS.  Step k forms
// eta = sum_{i <= k} col[k + 1 - i] a_k[i] (a workgroup reduction), then
// a_{k+1} = [a_k; 0] - (eta / err_k) [0; J conj(a_k)] in place, the pair
// (i, k + 1 - i) updated by one lane, and err_{k+1} = err_k - |eta|^2 / err_k.
// x_b = a_{L-1} / err_{L-1}.  status[b] = 0, or 1 if a pivot err_k is not
// positive (x_b then unspecified).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace fbst {

namespace {

constexpr int kLevThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int LMAX>
__global__ __launch_bounds__(kLevThreads) void k_levinson(const cx<double>* __restrict__ cols,
                                                          cx<double>* __restrict__ x,
                                                          int* __restrict__ status, int L) {
  __shared__ cx<double> a[LMAX];
  __shared__ double part[2][kLevThreads / 64];
  const int b = blockIdx.x, tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const cx<double>* col = cols + static_cast<size_t>(b) * L;
  for (int i = tid; i < L; i += kLevThreads) a[i] = cx<double>{i == 0 ? 1.0 : 0.0, 0.0};
  double err = col[0].re;
  bool ok = err > 0.0;
  __syncthreads();
  for (int k = 0; ok && k + 1 < L; ++k) {
    double er = 0.0, ei = 0.0;
    for (int i = tid; i <= k; i += kLevThreads) {
      const cx<double> c = col[k + 1 - i], ai = a[i];
      er += c.re * ai.re - c.im * ai.im;
      ei += c.re * ai.im + c.im * ai.re;
    }
    er = wave_sum(er);
    ei = wave_sum(ei);
    if (lane == 0) {
      part[0][wave] = er;
      part[1][wave] = ei;
    }
    __syncthreads();
    // every lane sums the wave partials in the same order: eta, g and err are
    // identical across the workgroup, so the loop exit is uniform
    double etr = 0.0, eti = 0.0;
#pragma unroll
    for (int w = 0; w < kLevThreads / 64; ++w) {
      etr += part[0][w];
      eti += part[1][w];
    }
    const double gr = etr / err, gi = eti / err;
    const int n = k + 1;
    for (int i = tid; i <= n - i; i += kLevThreads) {
      const int j = n - i;
      const cx<double> ai = a[i], aj = a[j];
      // a[i] - g conj(a[j]); a[j] - g conj(a[i])
      a[i] = cx<double>{ai.re - (gr * aj.re + gi * aj.im), ai.im - (gi * aj.re - gr * aj.im)};
      if (i != j)
        a[j] = cx<double>{aj.re - (gr * ai.re + gi * ai.im), aj.im - (gi * ai.re - gr * ai.im)};
    }
    err -= gr * etr + gi * eti;                // Re(g conj(eta))
    ok = err > 0.0;
    __syncthreads();
  }
  cx<double>* xb = x + static_cast<size_t>(b) * L;
  for (int i = tid; i < L; i += kLevThreads)
    xb[i] = ok ? cx<double>{a[i].re / err, a[i].im / err} : cx<double>{0.0, 0.0};
  if (tid == 0) status[b] = ok ? 0 : 1;
}

}  // namespace

hipError_t launch_levinson(const void* cols, void* x, int* status, int B, int L, hipStream_t st) {
  if (B < 1 || L < 1 || L > 8192 || !cols || !x || !status) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(B)), block(kLevThreads);
  if (L <= 4096)
    hipLaunchKernelGGL(k_levinson<4096>, grid, block, 0, st, static_cast<const cx<double>*>(cols),
                       static_cast<cx<double>*>(x), status, L);
  else
    hipLaunchKernelGGL(k_levinson<8192>, grid, block, 0, st, static_cast<const cx<double>*>(cols),
                       static_cast<cx<double>*>(x), status, L);
  return hipGetLastError();
}

}  // namespace fbst
