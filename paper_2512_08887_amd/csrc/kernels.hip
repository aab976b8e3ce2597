// HIP kernels of the FBST hot path for gfx950.
//
//   K1 stage 1a  time chirp-z per sensor          (Sec. IV, sum over n of eq. DFT_1)
//   K2 stage 1b  space chirp-z per frequency l     (Sec. IV, sum over m; App. B per axis)
//   K3 stage 2   Gohberg-Semencul Toeplitz apply + F_u chirp-z per beam (Sec. V)
//
// Every chirp-z is a Bluestein convolution held entirely in one workgroup:
// chirp premultiply while loading, forward FFT in LDS, product with the
// precomputed kernel spectrum in registers, inverse FFT, postmultiply while
// storing, so each operand crosses HBM once per stage.
#include <hip/hip_runtime.h>

#include "fft_lds.h"
#include "kernels.h"

namespace fbst {

namespace {

constexpr int kE = 16;          // elements per thread in every transform

template <int P>
struct Shape {
  static constexpr int TT = P / kE;                        // threads per transform
  static constexpr int G = (TT >= 256) ? 1 : 256 / TT;     // transforms per workgroup
  static constexpr int THREADS = TT * G;
  static constexpr int S = lds_stride(P);                  // LDS elements per transform
};

template <typename T>
__device__ __forceinline__ cx<T> ldg(const cx<T>* p) { return *p; }

// ---------------------------------------------------------------------------
// K1: Yhat[row][i] = post[i] * IFFT(FFT(x[row][n] * pre[n]) * H)[i],  i < L.
// rows are (block, sensor) pairs; lane = g * TT + t (a transform owns a
// contiguous run of lanes, so row loads and stores are coalesced).
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ __launch_bounds__(Shape<P>::THREADS) void k_time_czt(
    const cx<T>* __restrict__ x, cx<T>* __restrict__ yhat, const cx<T>* __restrict__ pre,
    const cx<T>* __restrict__ H, const cx<T>* __restrict__ post, const cx<T>* __restrict__ tw,
    int N, int L, int rows) {
  using SH = Shape<P>;
  __shared__ cx<T> lds[SH::G * SH::S];
  const int g = threadIdx.x / SH::TT;
  const int t = threadIdx.x % SH::TT;
  const int row = blockIdx.x * SH::G + g;
  const bool active = row < rows;
  cx<T>* buf = lds + g * SH::S;

  cx<T> v[kE];
  const cx<T>* src = x + static_cast<size_t>(row) * N;
#pragma unroll
  for (int s = 0; s < kE; ++s) {
    const int n = t + s * SH::TT;
    v[s] = (active && n < N) ? cmul(ldg(src + n), ldg(pre + n)) : cx<T>{0, 0};
  }
  fft<T, P, kE, -1>(v, buf, tw, t);
#pragma unroll
  for (int s = 0; s < kE; ++s) v[s] = cmul(v[s], ldg(H + t + s * SH::TT));
  fft<T, P, kE, +1>(v, buf, tw, t);
  cx<T>* dst = yhat + static_cast<size_t>(row) * L;
#pragma unroll
  for (int s = 0; s < kE; ++s) {
    const int i = t + s * SH::TT;
    if (active && i < L) dst[i] = cmul(v[s], ldg(post + i));
  }
}

// ---------------------------------------------------------------------------
// K2: one axis of the space chirp-z.  Data layout [blk][pre_n][A][post_n][L]
// (A = a_in on input, a_out on output); a workgroup takes G consecutive l for
// one (blk, p, q) and lane = t * G + g, so lanes with the same t read G
// consecutive l of one element.  Tables are l-fastest: pre [a_in][L],
// H [P][L], post [a_out][L].
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ __launch_bounds__(Shape<P>::THREADS) void k_axis_czt(
    const cx<T>* __restrict__ in, cx<T>* __restrict__ out, const cx<T>* __restrict__ pre,
    const cx<T>* __restrict__ H, const cx<T>* __restrict__ post, const cx<T>* __restrict__ tw,
    int a_in, int a_out, int pre_n, int post_n, int L, int n_tiles) {
  using SH = Shape<P>;
  __shared__ cx<T> lds[SH::G * SH::S];
  const int g = threadIdx.x % SH::G;
  const int t = threadIdx.x / SH::G;
  int wg = blockIdx.x;
  const int tile = wg % n_tiles;
  wg /= n_tiles;
  const int q = wg % post_n;
  wg /= post_n;
  const int p = wg % pre_n;
  const int blk = wg / pre_n;
  const int l = tile * SH::G + g;
  const bool active = l < L;
  cx<T>* buf = lds + g * SH::S;

  const size_t stride = static_cast<size_t>(post_n) * L;
  const cx<T>* src = in + ((static_cast<size_t>(blk) * pre_n + p) * a_in * post_n + q) * L + l;
  cx<T> v[kE];
#pragma unroll
  for (int s = 0; s < kE; ++s) {
    const int i = t + s * SH::TT;
    v[s] = (active && i < a_in) ? cmul(ldg(src + i * stride), ldg(pre + static_cast<size_t>(i) * L + l))
                                : cx<T>{0, 0};
  }
  fft<T, P, kE, -1>(v, buf, tw, t);
#pragma unroll
  for (int s = 0; s < kE; ++s) {
    const int i = t + s * SH::TT;
    v[s] = active ? cmul(v[s], ldg(H + static_cast<size_t>(i) * L + l)) : cx<T>{0, 0};
  }
  fft<T, P, kE, +1>(v, buf, tw, t);
  cx<T>* dst = out + ((static_cast<size_t>(blk) * pre_n + p) * a_out * post_n + q) * L + l;
#pragma unroll
  for (int s = 0; s < kE; ++s) {
    const int a = t + s * SH::TT;
    if (active && a < a_out) dst[a * stride] = cmul(v[s], ldg(post + static_cast<size_t>(a) * L + l));
  }
}

// ---------------------------------------------------------------------------
// K3: per beam, beta = A_b^{-1} w_b by the Gohberg-Semencul form
//   A^{-1} = (1/x0) [L(x) L(x)^H - L(y~) L(y~)^H],  y~ = (0, conj x_{L-1}, ..., conj x_1)
// with each triangular Toeplitz product done by circulant embedding in P
// points (G1 = FFT(x) and G2 = FFT(y~), both scaled by 1 / (P sqrt(x0))), then
// b = F_u beta as a Bluestein chirp-z in the same P points:
//   V = FFT(w);  p_k = IFFT(conj(G_k) V)[0:L];  Z = G1 FFT(p_1) - G2 FFT(p_2)
//   beta = IFFT(Z)[0:L];  b = post3 * IFFT(FFT(beta * pre3) * H3)[0:N]
// Eight P-point transforms, all in LDS/registers.
// ---------------------------------------------------------------------------
template <typename T, typename TIN, typename TOUT, int P>
__global__ __launch_bounds__(Shape<P>::THREADS) void k_toeplitz_fu(
    const cx<TIN>* __restrict__ w, cx<TOUT>* __restrict__ beams, const cx<T>* __restrict__ G1,
    const cx<T>* __restrict__ G2, const cx<T>* __restrict__ pre3, const cx<T>* __restrict__ H3,
    const cx<T>* __restrict__ post3, const cx<T>* __restrict__ tw, int B, int L, int N, int rows) {
  using SH = Shape<P>;
  __shared__ cx<T> lds[SH::G * SH::S];
  const int g = threadIdx.x / SH::TT;
  const int t = threadIdx.x % SH::TT;
  const int row = blockIdx.x * SH::G + g;
  const bool active = row < rows;
  const int b = active ? row % B : 0;
  cx<T>* buf = lds + g * SH::S;
  const cx<T>* g1 = G1 + static_cast<size_t>(b) * P;
  const cx<T>* g2 = G2 + static_cast<size_t>(b) * P;

  cx<T> V[kE];
  const cx<TIN>* src = w + static_cast<size_t>(row) * L;
#pragma unroll
  for (int s = 0; s < kE; ++s) {
    const int i = t + s * SH::TT;
    V[s] = (active && i < L) ? cvt<T>(src[i]) : cx<T>{0, 0};
  }
  fft<T, P, kE, -1>(V, buf, tw, t);

  cx<T> Z[kE];
  cx<T> u[kE];
  // branch 1: Z = G1 * FFT(trunc_L(IFFT(conj(G1) V)))
#pragma unroll
  for (int s = 0; s < kE; ++s) u[s] = cmulc(V[s], ldg(g1 + t + s * SH::TT));
  fft<T, P, kE, +1>(u, buf, tw, t);
#pragma unroll
  for (int s = 0; s < kE; ++s)
    if (t + s * SH::TT >= L) u[s] = cx<T>{0, 0};
  fft<T, P, kE, -1>(u, buf, tw, t);
#pragma unroll
  for (int s = 0; s < kE; ++s) Z[s] = cmul(u[s], ldg(g1 + t + s * SH::TT));
  // branch 2: Z -= G2 * FFT(trunc_L(IFFT(conj(G2) V)))
#pragma unroll
  for (int s = 0; s < kE; ++s) u[s] = cmulc(V[s], ldg(g2 + t + s * SH::TT));
  fft<T, P, kE, +1>(u, buf, tw, t);
#pragma unroll
  for (int s = 0; s < kE; ++s)
    if (t + s * SH::TT >= L) u[s] = cx<T>{0, 0};
  fft<T, P, kE, -1>(u, buf, tw, t);
#pragma unroll
  for (int s = 0; s < kE; ++s) Z[s] = Z[s] - cmul(u[s], ldg(g2 + t + s * SH::TT));
  // beta = trunc_L(IFFT(Z)), then the F_u chirp-z
  fft<T, P, kE, +1>(Z, buf, tw, t);
#pragma unroll
  for (int s = 0; s < kE; ++s) {
    const int i = t + s * SH::TT;
    Z[s] = (i < L) ? cmul(Z[s], ldg(pre3 + i)) : cx<T>{0, 0};
  }
  fft<T, P, kE, -1>(Z, buf, tw, t);
#pragma unroll
  for (int s = 0; s < kE; ++s) Z[s] = cmul(Z[s], ldg(H3 + t + s * SH::TT));
  fft<T, P, kE, +1>(Z, buf, tw, t);
  cx<TOUT>* dst = beams + static_cast<size_t>(row) * N;
#pragma unroll
  for (int s = 0; s < kE; ++s) {
    const int n = t + s * SH::TT;
    if (active && n < N) dst[n] = cvt<TOUT>(cmul(Z[s], ldg(post3 + n)));
  }
}

template <int P>
int grid_for(int rows) { return (rows + Shape<P>::G - 1) / Shape<P>::G; }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers: dispatch the runtime FFT size to the compiled instances.
// ---------------------------------------------------------------------------
#define FBST_FOR_EACH_P(X) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(8192) X(16384)

template <typename T>
hipError_t launch_time_czt(int P, const void* x, void* yhat, const void* pre, const void* H,
                           const void* post, const void* tw, int N, int L, int rows,
                           hipStream_t st) {
  switch (P) {
#define CASE(PP)                                                                             \
  case PP:                                                                                   \
    if constexpr (sizeof(T) * 2 * lds_stride(PP) <= 160 * 1024) {                            \
      hipLaunchKernelGGL((k_time_czt<T, PP>), dim3(grid_for<PP>(rows)), dim3(Shape<PP>::THREADS), \
                         0, st, (const cx<T>*)x, (cx<T>*)yhat, (const cx<T>*)pre,             \
                         (const cx<T>*)H, (const cx<T>*)post, (const cx<T>*)tw, N, L, rows);  \
      return hipGetLastError();                                                              \
    }                                                                                        \
    break;
    FBST_FOR_EACH_P(CASE)
#undef CASE
    default:
      break;
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_axis_czt(int P, const void* in, void* out, const void* pre, const void* H,
                           const void* post, const void* tw, int a_in, int a_out, int pre_n,
                           int post_n, int L, int nblocks, hipStream_t st) {
  switch (P) {
#define CASE(PP)                                                                             \
  case PP:                                                                                   \
    if constexpr (sizeof(T) * 2 * lds_stride(PP) <= 160 * 1024) {                            \
      const int n_tiles = (L + Shape<PP>::G - 1) / Shape<PP>::G;                             \
      const long long grid = 1LL * nblocks * pre_n * post_n * n_tiles;                       \
      if (grid <= 0 || grid > 0x7fffffffLL) return hipErrorInvalidValue;                    \
      hipLaunchKernelGGL((k_axis_czt<T, PP>), dim3((unsigned)grid), dim3(Shape<PP>::THREADS), 0, \
                         st, (const cx<T>*)in, (cx<T>*)out, (const cx<T>*)pre,               \
                         (const cx<T>*)H, (const cx<T>*)post, (const cx<T>*)tw, a_in, a_out,  \
                         pre_n, post_n, L, n_tiles);                                         \
      return hipGetLastError();                                                              \
    }                                                                                        \
    break;
    FBST_FOR_EACH_P(CASE)
#undef CASE
    default:
      break;
  }
  return hipErrorInvalidValue;
}

template <typename T, typename TIN, typename TOUT>
hipError_t launch_toeplitz_fu(int P, const void* w, void* beams, const void* G1, const void* G2,
                              const void* pre3, const void* H3, const void* post3, const void* tw,
                              int B, int L, int N, int rows, hipStream_t st) {
  switch (P) {
#define CASE(PP)                                                                             \
  case PP:                                                                                   \
    if constexpr (sizeof(T) * 2 * lds_stride(PP) <= 160 * 1024) {                            \
      hipLaunchKernelGGL((k_toeplitz_fu<T, TIN, TOUT, PP>), dim3(grid_for<PP>(rows)),         \
                         dim3(Shape<PP>::THREADS), 0, st, (const cx<TIN>*)w, (cx<TOUT>*)beams, \
                         (const cx<T>*)G1, (const cx<T>*)G2, (const cx<T>*)pre3,              \
                         (const cx<T>*)H3, (const cx<T>*)post3, (const cx<T>*)tw, B, L, N, rows); \
      return hipGetLastError();                                                              \
    }                                                                                        \
    break;
    FBST_FOR_EACH_P(CASE)
#undef CASE
    default:
      break;
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_time_czt<float>(int, const void*, void*, const void*, const void*,
                                           const void*, const void*, int, int, int, hipStream_t);
template hipError_t launch_time_czt<double>(int, const void*, void*, const void*, const void*,
                                            const void*, const void*, int, int, int, hipStream_t);
template hipError_t launch_axis_czt<float>(int, const void*, void*, const void*, const void*,
                                           const void*, const void*, int, int, int, int, int, int,
                                           hipStream_t);
template hipError_t launch_axis_czt<double>(int, const void*, void*, const void*, const void*,
                                            const void*, const void*, int, int, int, int, int, int,
                                            hipStream_t);
template hipError_t launch_toeplitz_fu<float, float, float>(int, const void*, void*, const void*,
                                                            const void*, const void*, const void*,
                                                            const void*, const void*, int, int,
                                                            int, int, hipStream_t);
template hipError_t launch_toeplitz_fu<double, float, float>(int, const void*, void*, const void*,
                                                             const void*, const void*, const void*,
                                                             const void*, const void*, int, int,
                                                             int, int, hipStream_t);
template hipError_t launch_toeplitz_fu<double, double, double>(int, const void*, void*, const void*,
                                                               const void*, const void*,
                                                               const void*, const void*,
                                                               const void*, int, int, int, int,
                                                               hipStream_t);

}  // namespace fbst
