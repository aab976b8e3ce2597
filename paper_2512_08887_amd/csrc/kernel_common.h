// Shared by the HIP kernel sources: tuning knobs, workgroup shapes,
// XCD-aware workgroup numbering and table-load helpers.
#pragma once

#include <hip/hip_runtime.h>

#include "fft_lds.h"
#include "kernels.h"


#ifndef FBST_K3_DUAL
#define FBST_K3_DUAL 1            // run the two Gohberg-Semencul branches as one dual FFT
#endif
#ifndef FBST_K3_WAVES
#define FBST_K3_WAVES 2           // minimum waves per SIMD the register allocation must allow
#endif
// Twiddle modes of the transforms (TwiddleMode in fft_lds.h), per kernel.
#ifndef FBST_K12_TW
#define FBST_K12_TW 1             // stages 1a and 1b: prefetched across barriers
#endif
#ifndef FBST_K3_TW
#define FBST_K3_TW 1              // stage 2, single transforms
#endif
#ifndef FBST_K3_TW_DUAL
#define FBST_K3_TW_DUAL 0         // stage 2, dual transforms
#endif
#ifndef FBST_K12_WAVES
#define FBST_K12_WAVES 0
#endif
#if FBST_K3_WAVES > 0
#define FBST_K3_ATTR __attribute__((amdgpu_waves_per_eu(FBST_K3_WAVES)))
#else
#define FBST_K3_ATTR
#endif
#if FBST_K12_WAVES > 0
#define FBST_K12_ATTR __attribute__((amdgpu_waves_per_eu(FBST_K12_WAVES)))
#else
#define FBST_K12_ATTR
#endif

namespace fbst {

namespace {

constexpr int kE = FFT_E;
constexpr int kXCD = 8;          // XCDs of an MI355X; workgroups are dealt round-robin

template <int P, int WG = 256>
struct Shape {
  static constexpr int TT = P / kE;                        // threads per transform
  static constexpr int G = (TT >= WG) ? 1 : WG / TT;       // transforms per workgroup
  static constexpr int THREADS = TT * G;
  static constexpr int S = lds_stride(P);                  // LDS elements per transform
};

#ifndef FBST_K2_THREADS
#define FBST_K2_THREADS 512       // workgroup size of the space chirp-z (frequencies per tile x TT)
#endif
template <int P>
using ShapeK2 = Shape<P, FBST_K2_THREADS>;

// Logical index of this workgroup such that the workgroups the hardware
// sends to one XCD (blockIdx % 8) form a contiguous logical range.
__device__ __forceinline__ int xcd_linear(int nwg) {
  const int b = blockIdx.x;
  const int x = b % kXCD, i = b / kXCD;
  const int q = nwg / kXCD, r = nwg % kXCD;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

template <typename T>
__device__ __forceinline__ cx<T> ldg(const cx<T>* p) { return *p; }

#ifndef FBST_BATCH
#define FBST_BATCH 1              // issue each group of independent table/data loads together
#endif

// Loads above this point are issued before anything below it (an empty asm
// statement with a memory clobber).  The register-pressure-driven scheduler
// otherwise places each table load right before its use, one L2 round trip
// after another; batched, their latencies overlap.
template <bool ON = FBST_BATCH>
__device__ __forceinline__ void issue_fence() {
  if constexpr (ON) asm volatile("" ::: "memory");
}

#ifndef FBST_K3_GB
#define FBST_K3_GB 16             // stage-2 spectrum loads issued this many at a time (0: as used)
#endif

// use(s, a[s], b[s]) for s < N, where a[s] = A[s * TT] and b[s] = B[s * TT]
// (B may be null: then b[s] is unused), loading GB slots at a time.
template <int GB, int N, int TT, typename T, typename Use>
__device__ __forceinline__ void with_tables(const cx<T>* __restrict__ A, const cx<T>* __restrict__ B,
                                            Use&& use) {
  if constexpr (GB <= 0) {
#pragma unroll
    for (int s = 0; s < N; ++s) use(s, ldg(A + s * TT), B ? ldg(B + s * TT) : cx<T>{0, 0});
  } else {
    static_assert(N % GB == 0, "group size must divide the slot count");
#pragma unroll
    for (int s0 = 0; s0 < N; s0 += GB) {
      cx<T> a[GB], b[GB];
#pragma unroll
      for (int i = 0; i < GB; ++i) {
        a[i] = ldg(A + (s0 + i) * TT);
        if (B) b[i] = ldg(B + (s0 + i) * TT);
      }
      issue_fence<true>();
#pragma unroll
      for (int i = 0; i < GB; ++i) use(s0 + i, a[i], b[i]);
    }
  }
}

template <int P>
int grid_for(int rows) { return (rows + Shape<P>::G - 1) / Shape<P>::G; }

// smallest of {E/4, E/2, E} slots covering n elements of a P-point transform
template <int P>
int slots_for(int n) {
  const int tt = Shape<P>::TT;
  const int s = (n + tt - 1) / tt;
  return s <= kE / 4 ? kE / 4 : (s <= kE / 2 ? kE / 2 : kE);
}

template <typename T, int P, int NBUF = 1>
constexpr bool fits_lds() { return sizeof(T) * 2 * lds_stride(P) * NBUF * Shape<P>::G <= 160 * 1024; }

// p itself, opaque to the optimiser (an empty asm that may change it), so
// that nothing computed from it is reused across the point of the call.
template <typename Q>
__device__ __forceinline__ Q* fresh(Q* p) {
  asm volatile("" : "+s"(p));
  return p;
}

// W^i = exp(-2 pi j i / P) for 0 <= i < P/2, from the twiddles of the last
// pass of a P-point transform (entries exp(-2 pi j k / P), k < P / R_last).
template <int P, typename T>
__device__ __forceinline__ cx<T> split_twiddle(const cx<T>* __restrict__ tw, int i) {
  constexpr int NSL = [] {
    int ns = 1;
    while (P / ns > kE) ns *= kE;
    return ns;
  }();
  constexpr int RL = P / NSL;
  static_assert(RL == 2 || RL == 4, "split twiddles need a last pass of radix 2 or 4");
  const cx<T>* base = tw + tw_offset(P, NSL);
  if constexpr (RL == 2) {
    return base[i];
  } else {
    const cx<T> v = base[i & (NSL - 1)];
    return (i >= NSL) ? rot90<-1>(v) : v;     // exp(-j pi / 2) exp(-2 pi j (i - NSL) / P)
  }
}

}  // namespace

#define FBST_FOR_EACH_P(X) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(8192) X(16384)

}  // namespace fbst
