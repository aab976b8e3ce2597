// Stage 1a (time chirp-z, Sec. IV) with its FFTs as blocked DFT contractions
// on the gfx950 matrix cores, in bfloat16 or float16 with split-precision
// compensation and float32 accumulation.
//
// The Bluestein structure is the one of the float32 kernel: chirp-premultiply,
// P-point FFT, product with the kernel spectrum, inverse FFT, postmultiply.
// Each radix-16 Stockham pass (the same passes, spans and twiddle tables as
// fft_lds.h) is a matrix product: the 16-point DFT of 16 butterflies is
//     [Y_re; Y_im] = [[W_re, -W_im], [W_im, W_re]] [X_re; X_im]   (32 x 32 real),
// done as v_mfma_f32_16x16x32 (16 outputs x 16 butterflies x 32 inputs) per
// part.  Operands are split a = a_hi + a_lo in the 16-bit type and the
// products a_hi b_hi + a_hi b_lo + a_lo b_hi are accumulated in float32
// (the lo x lo term is below float32 rounding).  Twiddles, the pointwise
// products and the remainder pass (P not a power of 16) stay in float32 on
// the vector units.  Data live in LDS in float32 between passes.
#include <hip/hip_runtime.h>

#include "fft_lds.h"
#include "kernels.h"

namespace fbst {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename V8>
struct Lo16;
template <>
struct Lo16<bf16x8> {
  using S = __bf16;
  static __device__ __forceinline__ f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Lo16<f16x8> {
  using S = _Float16;
  static __device__ __forceinline__ f32x4 mma(f16x8 a, f16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// x = hi + lo in the 16-bit type (lo is the rounding residue of hi)
template <typename V8>
__device__ __forceinline__ void split(float x, V8& hi, V8& lo, int e) {
  using S = typename Lo16<V8>::S;
  const S h = static_cast<S>(x);
  hi[e] = h;
  lo[e] = static_cast<S>(x - static_cast<float>(h));
}

// A operands of the real-embedded 16-point DFT for this lane:
// lane l holds row k = l % 16 and columns c = 8 (l / 16) + e of
//   A_re = [W_re | -W_im],  A_im = [W_im | W_re],  W[k][r] = exp(DIR j 2 pi k r / 16).
template <typename V8>
struct DftA {
  V8 re_hi, re_lo, im_hi, im_lo;
};

__device__ __forceinline__ float cos16(int m) {
  // cos(2 pi m / 16), m in [0, 16)
  const int q = m & 3;
  const float c[4] = {1.0f, static_cast<float>(detail::kC1), static_cast<float>(detail::kR2),
                      static_cast<float>(detail::kS1)};
  const int quad = m >> 2;               // angle = quad * pi/2 + q * pi/8
  const float cq = c[q], sq = (q == 0) ? 0.0f : c[4 - q];
  // cos(quad pi/2 + a) for quad = 0..3: cos a, -sin a, -cos a, sin a
  return quad == 0 ? cq : quad == 1 ? -sq : quad == 2 ? -cq : sq;
}

template <int DIR, typename V8>
__device__ __forceinline__ DftA<V8> make_dft_a(int lane) {
  DftA<V8> A;
  const int k = lane & 15;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int c = 8 * (lane >> 4) + e;
    const int r = c & 15;
    const int m = (k * r) & 15;
    const float wr = cos16(m);
    const float wi = DIR * cos16((m + 12) & 15);   // sin(x) = cos(x - pi/2)
    const float are = (c < 16) ? wr : -wi;
    const float aim = (c < 16) ? wi : wr;
    split(are, A.re_hi, A.re_lo, e);
    split(aim, A.im_hi, A.im_lo, e);
  }
  return A;
}

// One radix-16 Stockham pass (span NS) of a P-point transform on the matrix
// cores: wave w owns butterflies [64 w, 64 w + 64) as four tiles of 16.  In a
// tile, lane l carries butterfly j = tile + l % 16, inputs r = 8 ((l/16) % 2)
// + e (e < 8) and the real (l < 32) or imaginary (l >= 32) parts; it receives
// outputs k' = 4 (l / 16) + e' (e' < 4) of butterfly j.
template <int P, int NS, int DIR, typename V8>
__device__ __forceinline__ void mfma_pass(c32* __restrict__ buf, const c32* __restrict__ tw,
                                          const DftA<V8>& A, int wave, int lane) {
  constexpr int R = 16;
  const int col = lane & 15;
  const int rblk = (lane >> 4) & 1;
  const bool imag = lane >= 32;
  f32x4 dre[4], dim[4];
#pragma unroll
  for (int ti = 0; ti < 4; ++ti) {
    const int j = wave * 64 + ti * 16 + col;
    const int k = j & (NS - 1);
    V8 bhi, blo;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int r = 8 * rblk + e;
      c32 v = buf[read_slot<P, R>(j, r)];
      if constexpr (NS > 1) {
        if (r > 0) v = cmul_dir<DIR>(v, tw[tw_offset(P, NS) + (r - 1) * NS + k]);
      }
      split(imag ? v.im : v.re, bhi, blo, e);
    }
    const f32x4 z = {0.f, 0.f, 0.f, 0.f};
    f32x4 a = Lo16<V8>::mma(A.re_hi, bhi, z);
    a = Lo16<V8>::mma(A.re_hi, blo, a);
    dre[ti] = Lo16<V8>::mma(A.re_lo, bhi, a);
    f32x4 b = Lo16<V8>::mma(A.im_hi, bhi, z);
    b = Lo16<V8>::mma(A.im_hi, blo, b);
    dim[ti] = Lo16<V8>::mma(A.im_lo, bhi, b);
  }
  __syncthreads();   // all operands of the pass have been read
#pragma unroll
  for (int ti = 0; ti < 4; ++ti) {
    const int j = wave * 64 + ti * 16 + col;
    const int k = j & (NS - 1);
    const int base = (j - k) * R + k;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int kk = 4 * (lane >> 4) + e;
      buf[write_slot<R, NS>(base, kk)] = c32{dre[ti][e], dim[ti][e]};
    }
  }
  __syncthreads();
}

template <int P, int NS, int DIR, typename V8>
__device__ __forceinline__ void mfma_passes(c32* buf, const c32* tw, const DftA<V8>& A, int wave,
                                            int lane, int t) {
  constexpr int REM = P / NS;
  if constexpr (REM >= 16) {
    mfma_pass<P, NS, DIR>(buf, tw, A, wave, lane);
    if constexpr (REM > 16) mfma_passes<P, NS * 16, DIR>(buf, tw, A, wave, lane, t);
  } else {
    // remainder radix (P = 16^a * REM): one float32 Stockham pass through LDS
    c32 unused[FFT_E];
    PassTw<float, P, FFT_E, NS> none;
    stockham_pass<float, P, FFT_E, REM, NS, DIR, false, false, FFT_E, TW_LAZY>(unused, buf, buf, none,
                                                                            tw, t, [] {});
  }
}

// K1 with matrix-core FFTs.  One sensor row per workgroup of P / 16 threads
// (P >= 1024, so every wave is full); rows are (block, sensor) pairs.
template <int P, typename V8>
__global__ __launch_bounds__(P / FFT_E) void k_time_czt_mfma(
    const InPtrs xs, c32* __restrict__ yhat, const c32* __restrict__ pre,
    const c32* __restrict__ H, const c32* __restrict__ post, const c32* __restrict__ tw, int M,
    int N, int L) {
  constexpr int TT = P / FFT_E;
  static_assert(TT % 64 == 0, "matrix-core passes need full waves");
  __shared__ c32 buf[lds_stride(P)];
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int row = blockIdx.x;
  const int blk = row / M;
  const c32* src = static_cast<const c32*>(xs.p[blk]) + (row - blk * M) * (xs.ld > 0 ? xs.ld : N);
  const DftA<V8> Af = make_dft_a<-1, V8>(lane);
  const DftA<V8> Ai = make_dft_a<+1, V8>(lane);
  {
    // loads at clamped indices, issued together (empty asm with a memory
    // clobber), then the select; see the float32 kernels
    c32 xa[FFT_E], pa[FFT_E];
#pragma unroll
    for (int s = 0; s < FFT_E; ++s) {
      const int n = t + s * TT;
      const int nc = n < N ? n : N - 1;
      xa[s] = src[nc];
      pa[s] = pre[nc];
    }
    asm volatile("" ::: "memory");
#pragma unroll
    for (int s = 0; s < FFT_E; ++s) {
      const int n = t + s * TT;
      buf[lds_pad(n)] = (n < N) ? cmul(xa[s], pa[s]) : c32{0.f, 0.f};
    }
  }
  __syncthreads();
  mfma_passes<P, 1, -1>(buf, tw, Af, wave, lane, t);
  {
    c32 h[FFT_E];
#pragma unroll
    for (int s = 0; s < FFT_E; ++s) h[s] = H[t + s * TT];
    asm volatile("" ::: "memory");
#pragma unroll
    for (int s = 0; s < FFT_E; ++s) {
      const int i = t + s * TT;
      buf[lds_pad(i)] = cmul(buf[lds_pad(i)], h[s]);
    }
  }
  __syncthreads();
  mfma_passes<P, 1, +1>(buf, tw, Ai, wave, lane, t);
  c32* dst = yhat + static_cast<size_t>(row) * L;
  c32 po[FFT_E];
#pragma unroll
  for (int s = 0; s < FFT_E; ++s) {
    const int i = t + s * TT;
    po[s] = post[i < L ? i : L - 1];
  }
  asm volatile("" ::: "memory");
#pragma unroll
  for (int s = 0; s < FFT_E; ++s) {
    const int i = t + s * TT;
    if (i < L) dst[i] = cmul(buf[lds_pad(i)], po[s]);
  }
}

}  // namespace

hipError_t launch_time_czt_mfma(int P, bool fp16, const InPtrs& xs, int nblocks, void* yhat,
                                const void* pre, const void* H, const void* post, const void* tw,
                                int M, int N, int L, hipStream_t st) {
  if (nblocks < 1 || nblocks > MAX_LAUNCH_BLOCKS) return hipErrorInvalidValue;
  const dim3 grid(nblocks * M);
  switch (P) {
#define CASE(PP)                                                                              \
  case PP:                                                                                    \
    if (fp16)                                                                                 \
      hipLaunchKernelGGL((k_time_czt_mfma<PP, f16x8>), grid, dim3(PP / FFT_E), 0, st, xs,     \
                         (c32*)yhat, (const c32*)pre, (const c32*)H, (const c32*)post,         \
                         (const c32*)tw, M, N, L);                                             \
    else                                                                                      \
      hipLaunchKernelGGL((k_time_czt_mfma<PP, bf16x8>), grid, dim3(PP / FFT_E), 0, st, xs,    \
                         (c32*)yhat, (const c32*)pre, (const c32*)H, (const c32*)post,         \
                         (const c32*)tw, M, N, L);                                             \
    return hipGetLastError();
    CASE(1024)
    CASE(2048)
    CASE(4096)
    CASE(8192)
    CASE(16384)
#undef CASE
    default:
      break;
  }
  return hipErrorInvalidValue;
}

}  // namespace fbst
