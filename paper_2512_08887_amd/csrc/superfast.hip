// Generators of the stage-2 Toeplitz systems on the GPU by the superfast
// doubling Schur algorithm (superfast.h): one workgroup per system, float64,
// the polynomial products by radix-2 FFTs in LDS, the recursion's windows and
// 2 x 2 polynomial matrices in a global scratch slot of the workgroup.  The
// grid holds at most one workgroup per compute unit (137 KB of LDS each);
// each takes systems blockIdx.x, blockIdx.x + gridDim.x, ... in turn.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "superfast.h"

namespace fbst {

namespace {

constexpr int kSfThreads = 256;
constexpr int kSfLMax = 4096;
// LDS elements for L <= kSfLMax: superfast::lds_elems(kSfLMax)
constexpr int kSfLds = 2 * kSfLMax + 2 * (2 * superfast::kBase + 4 * (superfast::kBase + 1));

// Ordering among the lanes of one wave: the wave's LDS operations complete in
// issue order, so a fence at wavefront scope (which keeps the compiler from
// moving memory operations across it) is all that work done by one wave
// needs between its steps.
__device__ __forceinline__ void wave_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct DevSync {
  __device__ void operator()() const { __syncthreads(); }
  __device__ void wave() const { wave_order(); }
};

struct WaveSync {
  __device__ void operator()() const { wave_order(); }
  __device__ void wave() const { wave_order(); }
};

__global__ __launch_bounds__(kSfThreads) void k_superfast(const cx<double>* __restrict__ cols,
                                                          cx<double>* __restrict__ x,
                                                          int* __restrict__ status, int B, int L,
                                                          cx<double>* __restrict__ scratch,
                                                          size_t per_wg,
                                                          const cx<double>* __restrict__ tw,
                                                          int PM) {
  __shared__ cx<double> lds[kSfLds];
  const superfast::Ctx c{static_cast<int>(threadIdx.x), static_cast<int>(blockDim.x), tw, PM};
  cx<double>* sc = scratch + static_cast<size_t>(blockIdx.x) * per_wg;
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    const size_t off = static_cast<size_t>(b) * L;
    // base cases (at most kBase steps on windows of at most kBase coefficients) on
    // the first wave alone, without workgroup barriers between their steps
    auto base = [&](const cx<double>* f, const cx<double>* g, int n, cx<double>* th,
                    cx<double>* buf) {
      if (threadIdx.x < 64) {
        const superfast::Ctx cw{static_cast<int>(threadIdx.x), 64, tw, PM};
        superfast::base_case(f, g, n, th, buf, cw, WaveSync{});
      }
      __syncthreads();
    };
    const bool ok = superfast::generator(cols + off, x + off, L, sc, lds, c, DevSync{}, base);
    if (threadIdx.x == 0) status[b] = ok ? 0 : 1;
    __syncthreads();
  }
}

}  // namespace

size_t superfast_scratch_bytes(int B, int L, int* grid) {
  int dev = 0, cus = 1;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 1;
  const int g = std::max(1, std::min(B, cus));
  if (grid) *grid = g;
  return static_cast<size_t>(g) * superfast::scratch_elems(L) * sizeof(cx<double>);
}

hipError_t launch_superfast(const void* cols, void* x, int* status, int B, int L, void* scratch,
                            size_t scratch_bytes, const void* tw, hipStream_t st) {
  if (B < 1 || L < 2 || L > kSfLMax || !cols || !x || !status || !scratch || !tw)
    return hipErrorInvalidValue;
  int grid = 0;
  if (superfast_scratch_bytes(B, L, &grid) > scratch_bytes) return hipErrorInvalidValue;
  const size_t per_wg = superfast::scratch_elems(L);
  hipLaunchKernelGGL(k_superfast, dim3(grid), dim3(kSfThreads), 0, st,
                     static_cast<const cx<double>*>(cols), static_cast<cx<double>*>(x), status, B,
                     L, static_cast<cx<double>*>(scratch), per_wg,
                     static_cast<const cx<double>*>(tw), superfast::max_fft(L));
  return hipGetLastError();
}

}  // namespace fbst
