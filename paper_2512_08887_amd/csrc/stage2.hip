// Stage 2 of the FBST hot path for gfx950 (K3): per beam, the Toeplitz solve
// of Sec. V by its Gohberg-Semencul form and F_u as a chirp-z transform,
// one workgroup per (block, beam) row, everything in LDS and registers.
#include "kernel_common.h"

#include <algorithm>

namespace fbst {

namespace {

// ---------------------------------------------------------------------------
// K3: per beam, beta = A_b^{-1} w_b by the Gohberg-Semencul form
//   A^{-1} = (1/x0) [L(x) L(x)^H - L(y~) L(y~)^H],  y~ = (0, conj x_{L-1}, ..., conj x_1)
// with each triangular Toeplitz product done by circulant embedding in P
// points (G1 = FFT(x) and G2 = FFT(y~), both scaled by 1 / (P sqrt(x0))), then
// b = F_u beta as a Bluestein chirp-z in the same P points:
//   V = FFT(w);  u_k = conj(G_k) V;  p_k = IFFT(u_k)[0:L]
//   Z = G1 FFT(p_1) - G2 FFT(p_2);  beta = IFFT(Z)[0:L]
//   b = post3 * IFFT(FFT(beta * pre3) * H3)[0:N]
// Eight P-point transforms, all in LDS/registers.  L <= P/2 always (P >= 2L - 1),
// so every L-long operand fills the first P/2 slots (SL = E/2); SN >= ceil(N / TT).
// Both products with V are formed at once so V is dead before the branches.
// Logical order: beam outermost, so the spectra of one beam are reused by the
// workgroups of all blocks on one XCD.
// ---------------------------------------------------------------------------
// Dual-branch stage 2 when two transforms of P points fit the LDS of a CU.
template <typename T, int P>
constexpr bool k3_two_buffers() {
  return sizeof(T) * 2 * lds_stride(P) * 2 * Shape<P>::G <= 160 * 1024;
}
template <typename T, int P>
constexpr bool k3_dual() {
  return FBST_K3_DUAL && k3_two_buffers<T, P>();
}
#ifndef FBST_K3_PING
#define FBST_K3_PING 1
#endif

// Stage 2 with one step of iterative refinement (MODE 1 then MODE 2, two
// launches): the float32 Gohberg-Semencul apply loses accuracy where its two
// terms, each much larger than beta, cancel; a second apply to the residual
// r = w - A beta_1 (A by circulant embedding of its first column, CA =
// FFT(c_0 .. c_{L-1}, 0 .., conj c_{L-1} .. conj c_1) / P) recovers it:
//   MODE 0  beta = GS(w); beams = F_u beta                       (8 transforms)
//   MODE 1  beta_1 = GS(w) stored to bt [rows][L]                (6 transforms)
//   MODE 2  r = w - A beta_1; beta = beta_1 + GS(r); beams = F_u beta (10 transforms)
// Instance variants, chosen at run time (fbst_autotune):
//   K3_SINGLE      the two Gohberg-Semencul branches one after the other, each
//                  transform alternating its exchanges between two buffers
//                  (default: the branches as one dual transform in two
//                  buffers, where they fit);
//   K3_PERSISTENT  a grid of at most the resident workgroups, each taking a
//                  contiguous range of rows (default: one workgroup per row
//                  group).
// The persistent grid runs the same per-row code, so its beams are bit-identical
// to the one-workgroup-per-row form; the single-buffer form rounds the
// combination of the two branches in another order (float32 rounding level).
constexpr int K3_SINGLE = 1;
constexpr int K3_PERSISTENT = 2;
constexpr int K3_WAVES3 = 4;     // registers for 3 waves per SIMD (single form, one buffer)

template <typename T, typename TIN, typename TOUT, int P, int SN, int MODE, bool DUAL, bool PING>
__device__ __forceinline__ void k3_row(
    int lw, cx<T>* __restrict__ lds, const cx<TIN>* __restrict__ w, const OutPtrs& outs,
    const cx<T>* __restrict__ G1, const cx<T>* __restrict__ G2, const cx<T>* __restrict__ pre3,
    const cx<T>* __restrict__ H3, const cx<T>* __restrict__ post3, const cx<T>* __restrict__ tw,
    int B, int L, int N, int nblocks, cx<T>* __restrict__ bt, const cx<T>* __restrict__ CA) {
  using SH = Shape<P>;
  constexpr int SL = kE / 2;
  // PING: the single form alternates its transforms' exchanges between two
  // buffers (one barrier per exchange)
  constexpr int NBUF = (DUAL || PING) ? 2 : 1;
  const int g = threadIdx.x / SH::TT;
  const int t = threadIdx.x % SH::TT;
  const int rows = nblocks * B;
  const bool active = lw < rows;
  const int b = active ? lw / nblocks : 0;
  const int blk = active ? lw % nblocks : 0;
  const size_t row = static_cast<size_t>(blk) * B + b;
  cx<T>* buf = lds + g * NBUF * SH::S;
  const cx<T>* g1 = G1 + static_cast<size_t>(b) * P;
  const cx<T>* g2 = G2 + static_cast<size_t>(b) * P;

  cx<T> u1[kE], u2[kE];
  const cx<TIN>* src = w + row * L;                   // row of block 0, beam 0 when inactive
  cx<T>* brow = bt + row * L;
  if constexpr (MODE == 2) {
    // r = w - A beta_1, A beta_1 = IFFT(CA FFT(beta_1)) (circulant embedding)
#pragma unroll
    for (int s = 0; s < kE; ++s) {
      const int i = t + s * SH::TT;
      u1[s] = (s < SL && active && i < L) ? brow[i] : cx<T>{0, 0};
    }
    fft<T, P, kE, -1, SL, FBST_K3_TW, PING>(u1, buf, tw, t);
    with_tables<FBST_K3_GB, kE, SH::TT>(CA + static_cast<size_t>(b) * P + t,
                                        static_cast<const cx<T>*>(nullptr),
                                        [&](int s, cx<T> a, cx<T>) { u1[s] = cmul(u1[s], a); });
    fft<T, P, kE, +1, kE, FBST_K3_TW, PING>(u1, buf, tw, t);
#pragma unroll
    for (int s = 0; s < kE; ++s) {
      const int i = t + s * SH::TT;
      u1[s] = (s < SL && active && i < L) ? cvt<T>(src[i]) - u1[s] : cx<T>{0, 0};
    }
  } else {
#pragma unroll
    for (int s = 0; s < kE; ++s) {
      const int i = t + s * SH::TT;
      u1[s] = (s < SL && active && i < L) ? cvt<T>(src[i]) : cx<T>{0, 0};
    }
  }
  fft<T, P, kE, -1, SL, FBST_K3_TW, PING>(u1, buf, tw, t);
  with_tables<FBST_K3_GB, kE, SH::TT>(g1 + t, g2 + t, [&](int s, cx<T> a, cx<T> c) {
    const cx<T> V = u1[s];
    u1[s] = cmulc(V, a);
    u2[s] = cmulc(V, c);
  });
  if constexpr (DUAL) {
    // both branches: u_k <- FFT(trunc_L(IFFT(u_k)))
    fft2<T, P, kE, +1, kE, FBST_K3_TW_DUAL>(u1, u2, buf, buf + SH::S, tw, t);
#pragma unroll
    for (int s = 0; s < kE; ++s)
      if (s >= SL || t + s * SH::TT >= L) {
        u1[s] = cx<T>{0, 0};
        u2[s] = cx<T>{0, 0};
      }
    fft2<T, P, kE, -1, SL, FBST_K3_TW_DUAL>(u1, u2, buf, buf + SH::S, tw, t);
    with_tables<FBST_K3_GB, kE, SH::TT>(g1 + t, g2 + t, [&](int s, cx<T> a, cx<T> c) {
      u1[s] = cmul(u1[s], a) - cmul(u2[s], c);
    });
  } else {
    // branch 1: u1 <- G1 * FFT(trunc_L(IFFT(u1)))
    fft<T, P, kE, +1, kE, FBST_K3_TW, PING>(u1, buf, tw, t);
#pragma unroll
    for (int s = 0; s < kE; ++s)
      if (s >= SL || t + s * SH::TT >= L) u1[s] = cx<T>{0, 0};
    fft<T, P, kE, -1, SL, FBST_K3_TW, PING>(u1, buf, tw, t);
#pragma unroll
    for (int s = 0; s < kE; ++s) u1[s] = cmul(u1[s], ldg(g1 + t + s * SH::TT));
    // branch 2: u1 -= G2 * FFT(trunc_L(IFFT(u2)))
    fft<T, P, kE, +1, kE, FBST_K3_TW, PING>(u2, buf, tw, t);
#pragma unroll
    for (int s = 0; s < kE; ++s)
      if (s >= SL || t + s * SH::TT >= L) u2[s] = cx<T>{0, 0};
    fft<T, P, kE, -1, SL, FBST_K3_TW, PING>(u2, buf, tw, t);
#pragma unroll
    for (int s = 0; s < kE; ++s) u1[s] = u1[s] - cmul(u2[s], ldg(g2 + t + s * SH::TT));
  }
  // beta = trunc_L(IFFT(Z)), then the F_u chirp-z
  fft<T, P, kE, +1, kE, FBST_K3_TW, PING>(u1, buf, tw, t);
  if constexpr (MODE == 1) {
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const int i = t + s * SH::TT;
      if (active && i < L) brow[i] = u1[s];
    }
    return;
  }
  if constexpr (MODE == 2) {
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const int i = t + s * SH::TT;
      if (i < L) u1[s] = u1[s] + brow[active ? i : 0];
    }
  }
#pragma unroll
  for (int s = 0; s < kE; ++s) {
    const int i = t + s * SH::TT;
    u1[s] = (s < SL && i < L) ? cmul(u1[s], ldg(pre3 + i)) : cx<T>{0, 0};
  }
  fft<T, P, kE, -1, SL, FBST_K3_TW, PING>(u1, buf, tw, t);
  with_tables<FBST_K3_GB, kE, SH::TT>(H3 + t, static_cast<const cx<T>*>(nullptr),
                                      [&](int s, cx<T> a, cx<T>) { u1[s] = cmul(u1[s], a); });
  fft<T, P, kE, +1, kE, FBST_K3_TW, PING>(u1, buf, tw, t);
  cx<TOUT>* dst = static_cast<cx<TOUT>*>(outs.p[blk]) + static_cast<size_t>(b) * N;
#pragma unroll
  for (int s = 0; s < SN; ++s) {
    const int n = t + s * SH::TT;
    if (active && n < N) dst[n] = cvt<TOUT>(cmul(u1[s], ldg(post3 + n)));
  }
}

template <typename T, typename TIN, typename TOUT, int P, int SN, int MODE = 0, int VAR = 0>
__global__ __launch_bounds__(Shape<P>::THREADS)
__attribute__((amdgpu_waves_per_eu((VAR & K3_WAVES3) ? 3 : FBST_K3_WAVES))) void k_toeplitz_fu(
    const cx<TIN>* __restrict__ w, const OutPtrs outs, const cx<T>* __restrict__ G1,
    const cx<T>* __restrict__ G2, const cx<T>* __restrict__ pre3, const cx<T>* __restrict__ H3,
    const cx<T>* __restrict__ post3, const cx<T>* __restrict__ tw, int B, int L, int N,
    int nblocks, cx<T>* __restrict__ bt = nullptr, const cx<T>* __restrict__ CA = nullptr) {
  using SH = Shape<P>;
  constexpr bool DUAL = !(VAR & K3_SINGLE) && k3_dual<T, P>();
  // the single form takes two alternating buffers where they fit, except in
  // the instance that keeps its registers for 3 waves per SIMD (the second
  // buffer would leave room for two workgroups only)
  constexpr bool PING = FBST_K3_PING && !DUAL && !(VAR & K3_WAVES3) && k3_two_buffers<T, P>();
  __shared__ cx<T> lds[SH::G * ((DUAL || PING) ? 2 : 1) * SH::S];
  const int g = threadIdx.x / SH::TT;
  const int wl = xcd_linear(gridDim.x);                 // contiguous logical range per XCD
  if constexpr (VAR & K3_PERSISTENT) {
    // row groups [wl per, (wl + 1) per): the trip count is uniform in the
    // workgroup (its barriers are reached by every thread each time)
    const int groups = (nblocks * B + SH::G - 1) / SH::G;
    const int per = (groups + static_cast<int>(gridDim.x) - 1) / static_cast<int>(gridDim.x);
    const int q1 = min(groups, (wl + 1) * per);
    for (int q = wl * per; q < q1; ++q)
      k3_row<T, TIN, TOUT, P, SN, MODE, DUAL, PING>(q * SH::G + g, lds, w, outs, G1, G2, pre3, H3, post3,
                                              tw, B, L, N, nblocks, bt, CA);
  } else {
    k3_row<T, TIN, TOUT, P, SN, MODE, DUAL, PING>(wl * SH::G + g, lds, w, outs, G1, G2, pre3, H3, post3,
                                            tw, B, L, N, nblocks, bt, CA);
  }
}

}  // namespace

// Stage 2 with one refinement step (float32): MODE 1 (beta_1 to bt) then
// MODE 2 (residual, correction, F_u), both of one launch shape.
hipError_t launch_toeplitz_fu_refined(int P, const void* w, const OutPtrs& outs, const void* G1,
                                      const void* G2, const void* pre3, const void* H3,
                                      const void* post3, const void* tw, const void* CA, void* bt,
                                      int B, int L, int N, int nblocks, hipStream_t st) {
  if (nblocks < 1 || nblocks > MAX_LAUNCH_BLOCKS || !CA || !bt) return hipErrorInvalidValue;
  using T = float;
  switch (P) {
#define CASE(PP)                                                                               \
  case PP: {                                                                                   \
    if (2 * L > PP) return hipErrorInvalidValue;                                               \
    const dim3 grid(grid_for<PP>(nblocks * B)), block(Shape<PP>::THREADS);                     \
    const int sn = slots_for<PP>(N);                                                           \
    const auto a = (const cx<T>*)w;                                                            \
    const auto& o = outs;                                                                      \
    const auto g1 = (const cx<T>*)G1, g2 = (const cx<T>*)G2, p3 = (const cx<T>*)pre3;          \
    const auto h3 = (const cx<T>*)H3, q3 = (const cx<T>*)post3, twp = (const cx<T>*)tw;        \
    const auto ca = (const cx<T>*)CA;                                                          \
    const auto b1 = (cx<T>*)bt;                                                                \
    hipLaunchKernelGGL((k_toeplitz_fu<T, T, T, PP, kE / 4, 1>), grid, block, 0, st, a, o, g1, g2, \
                       p3, h3, q3, twp, B, L, N, nblocks, b1, ca);                             \
    if (sn <= kE / 4)                                                                          \
      hipLaunchKernelGGL((k_toeplitz_fu<T, T, T, PP, kE / 4, 2>), grid, block, 0, st, a, o, g1,  \
                         g2, p3, h3, q3, twp, B, L, N, nblocks, b1, ca);                       \
    else if (sn <= kE / 2)                                                                     \
      hipLaunchKernelGGL((k_toeplitz_fu<T, T, T, PP, kE / 2, 2>), grid, block, 0, st, a, o, g1,  \
                         g2, p3, h3, q3, twp, B, L, N, nblocks, b1, ca);                       \
    else                                                                                       \
      hipLaunchKernelGGL((k_toeplitz_fu<T, T, T, PP, kE, 2>), grid, block, 0, st, a, o, g1, g2,  \
                         p3, h3, q3, twp, B, L, N, nblocks, b1, ca);                           \
    return hipGetLastError();                                                                  \
  }
    CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096) CASE(8192) CASE(16384)
#undef CASE
    default:
      break;
  }
  return hipErrorInvalidValue;
}

namespace {

// One launch of k_toeplitz_fu<.., PP, SNV, 0, VAR>; a persistent variant's
// grid is the number of workgroups resident at once (occupancy of this
// instance times the compute units), or fewer when there are fewer row groups.
template <typename T, typename TIN, typename TOUT, int PP, int SNV, int VAR>
hipError_t k3_launch(const void* w, const OutPtrs& outs, const void* G1, const void* G2,
                     const void* pre3, const void* H3, const void* post3, const void* tw, int B,
                     int L, int N, int nblocks, hipStream_t st) {
  int grid = grid_for<PP>(nblocks * B);
  if constexpr ((VAR & K3_PERSISTENT) != 0) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(&k_toeplitz_fu<T, TIN, TOUT, PP, SNV, 0, VAR>),
          Shape<PP>::THREADS, 0);
    if (e != hipSuccess) return e;
    grid = std::min(grid, std::max(1, cus * per_cu));
  }
  hipLaunchKernelGGL((k_toeplitz_fu<T, TIN, TOUT, PP, SNV, 0, VAR>), dim3(grid),
                     dim3(Shape<PP>::THREADS), 0, st, (const cx<TIN>*)w, outs, (const cx<T>*)G1,
                     (const cx<T>*)G2, (const cx<T>*)pre3, (const cx<T>*)H3, (const cx<T>*)post3,
                     (const cx<T>*)tw, B, L, N, nblocks, nullptr, nullptr);
  return hipGetLastError();
}

// Variants other than 0 are compiled for float32 stage 2 at P >= 1024.
template <typename T, int PP>
constexpr bool k3_has_variants() {
  return sizeof(T) == 4 && PP >= 1024;
}

template <typename T, typename TIN, typename TOUT, int PP, int SNV>
hipError_t k3_dispatch_var(int var, const void* w, const OutPtrs& outs, const void* G1,
                           const void* G2, const void* pre3, const void* H3, const void* post3,
                           const void* tw, int B, int L, int N, int nblocks, hipStream_t st) {
  if constexpr (k3_has_variants<T, PP>()) {
    switch (var) {
      case 1:
        return k3_launch<T, TIN, TOUT, PP, SNV, 1>(w, outs, G1, G2, pre3, H3, post3, tw, B, L, N,
                                                   nblocks, st);
      case 2:
        return k3_launch<T, TIN, TOUT, PP, SNV, 2>(w, outs, G1, G2, pre3, H3, post3, tw, B, L, N,
                                                   nblocks, st);
      case 3:
        return k3_launch<T, TIN, TOUT, PP, SNV, 3>(w, outs, G1, G2, pre3, H3, post3, tw, B, L, N,
                                                   nblocks, st);
      case 5:
        return k3_launch<T, TIN, TOUT, PP, SNV, 5>(w, outs, G1, G2, pre3, H3, post3, tw, B, L, N,
                                                   nblocks, st);
      default:
        break;
    }
  }
  if (var != 0) return hipErrorInvalidValue;
  return k3_launch<T, TIN, TOUT, PP, SNV, 0>(w, outs, G1, G2, pre3, H3, post3, tw, B, L, N,
                                             nblocks, st);
}

}  // namespace

bool k3_variant_available(int P, bool fp32_stage2, int var) {
  if (var == 0) return true;
  const bool compiled = (var >= 1 && var <= 3) || var == (K3_SINGLE | K3_WAVES3);
  return fp32_stage2 && compiled && P >= 1024 && P <= PMAX;
}

template <typename T, typename TIN, typename TOUT>
hipError_t launch_toeplitz_fu(int P, const void* w, const OutPtrs& outs, const void* G1,
                              const void* G2, const void* pre3, const void* H3, const void* post3,
                              const void* tw, int B, int L, int N, int nblocks, hipStream_t st,
                              int var) {
  if (nblocks < 1 || nblocks > MAX_LAUNCH_BLOCKS) return hipErrorInvalidValue;
  switch (P) {
#define CASE(PP)                                                                               \
  case PP:                                                                                     \
    if constexpr (fits_lds<T, PP>()) {                                                         \
      if (2 * L > PP) return hipErrorInvalidValue;                                             \
      const int sn = slots_for<PP>(N);                                                         \
      if (sn <= kE / 4)                                                                        \
        return k3_dispatch_var<T, TIN, TOUT, PP, kE / 4>(var, w, outs, G1, G2, pre3, H3, post3, \
                                                         tw, B, L, N, nblocks, st);            \
      if (sn <= kE / 2)                                                                        \
        return k3_dispatch_var<T, TIN, TOUT, PP, kE / 2>(var, w, outs, G1, G2, pre3, H3, post3, \
                                                         tw, B, L, N, nblocks, st);            \
      return k3_dispatch_var<T, TIN, TOUT, PP, kE>(var, w, outs, G1, G2, pre3, H3, post3, tw, B, \
                                                   L, N, nblocks, st);                         \
    }                                                                                          \
    break;
    FBST_FOR_EACH_P(CASE)
#undef CASE
    default:
      break;
  }
  return hipErrorInvalidValue;
}

namespace {

// ---------------------------------------------------------------------------
// Float64 stage 2 at P points when one float64 P-point transform exceeds the
// LDS (P = 16384: 256 KiB).  Each P-point transform becomes two H = P/2-point
// transforms in LDS with one radix-2 step in the registers around them
// (W = exp(-2 pi j / P), H-point index n, k):
//   forward, input zero at n >= H (every forward transform of stage 2, since
//   L <= P/2 and the F_u input is L long):
//     X[2k] = FFT_H(x)[k],   X[2k + 1] = FFT_H(x[n] W^n)[k];
//   inverse (unscaled):
//     x[n] = a[n] + W^-n b[n],  x[n + H] = a[n] - W^-n b[n],
//     a = IFFT_H(X[2k]), b = IFFT_H(X[2k + 1]).
// A spectrum is therefore held as [even half | odd half]; the products with
// G1, G2 and H3 read the natural-order tables at 2k and 2k + 1.  Between the
// transforms the two branch spectra of a row sit in a global scratch of
// [2][P] elements per workgroup; each element is written and read back by
// the same thread (slot s of thread t is element t + s TT of both halves), so
// the scratch needs no barrier.  The grid is at most kSplitGrid workgroups,
// each taking a contiguous range of rows.
// ---------------------------------------------------------------------------
// at most this many workgroups: one per CU (float64: 139 KiB of LDS)
template <typename T>
constexpr int split_grid() {
  return 256;
}
constexpr int kSplitTw = FBST_K3_TW;

template <typename T, typename TIN, typename TOUT, int P>
__global__ __launch_bounds__(Shape<P / 2>::THREADS) void k_toeplitz_fu_split(
    const cx<TIN>* __restrict__ w, const OutPtrs outs, const cx<T>* __restrict__ G1,
    const cx<T>* __restrict__ G2, const cx<T>* __restrict__ pre3,
    const cx<T>* __restrict__ H3, const cx<T>* __restrict__ post3,
    const cx<T>* __restrict__ twg, int B, int L, int N, int nblocks,
    cx<T>* __restrict__ scratch) {
  constexpr int H = P / 2;
  using SH = Shape<H>;
  static_assert(SH::G == 1, "one half transform per workgroup");
  constexpr int TT = SH::TT;
  __shared__ cx<T> lds[SH::S];
  const int t = threadIdx.x;
  const int wl = xcd_linear(gridDim.x);
  cx<T>* const U1w = scratch + static_cast<size_t>(wl) * 2 * P;
  const int rows = nblocks * B;
  const int per = (rows + static_cast<int>(gridDim.x) - 1) / static_cast<int>(gridDim.x);
  const int r1 = min(rows, (wl + 1) * per);
  cx<T> v[kE];
  // One half transform is live in registers at a time; the other half waits
  // in the scratch.  Each loop below takes its base pointers through fresh():
  // the compiler then recomputes the per-slot addresses (and reloads table
  // values) where they are used instead of keeping those of every array live
  // across the transforms, which spills.
  auto load = [&](const cx<T>* a) {
    a = fresh(a);
#pragma unroll
    for (int s = 0; s < kE; ++s) v[s] = a[t + s * TT];
  };
  auto store = [&](cx<T>* a) {
    a = fresh(a);
#pragma unroll
    for (int s = 0; s < kE; ++s) a[t + s * TT] = v[s];
  };
  // (the thread index too goes through an empty asm per transform, so that
  // the LDS addresses of the passes are not kept live between transforms)
  auto fwd = [&] {
    int tf = t;
    asm volatile("" : "+v"(tf));
    fft<T, H, kE, -1, kE, kSplitTw>(v, lds, fresh(twg), tf);
  };
  auto inv = [&] {
    int tf = t;
    asm volatile("" : "+v"(tf));
    fft<T, H, kE, +1, kE, kSplitTw>(v, lds, fresh(twg), tf);
  };
  // every thread runs the same trip count (the transforms hold barriers)
  for (int row = wl * per; row < r1; ++row) {
    cx<T>* const U1 = U1w;                               // Z accumulates here
    cx<T>* const U2 = U1w + P;
    const int bm = row / nblocks, blk = row % nblocks;
    const cx<TIN>* const src = w + (static_cast<size_t>(blk) * B + bm) * L;
    const cx<T>* const g1 = G1 + static_cast<size_t>(bm) * P;
    const cx<T>* const g2 = G2 + static_cast<size_t>(bm) * P;

    // V = FFT_P(w); U1 = conj(G1) V, U2 = conj(G2) V
#pragma unroll 1
    for (int par = 0; par < 2; ++par) {
      {
        const cx<TIN>* x0 = fresh(src);
        const cx<T>* tw = fresh(twg);
#pragma unroll
        for (int s = 0; s < kE; ++s) {
          const int i = t + s * TT;
          const cx<T> x = (i < L) ? cvt<T>(x0[i]) : cx<T>{0, 0};
          v[s] = par ? cmul(x, split_twiddle<P>(tw, i)) : x;
          issue_fence<true>();   // bound the loads in flight
        }
      }
      fwd();
      cx<T>* u1 = fresh(U1);
      cx<T>* u2 = fresh(U2);
      const cx<T>* a1 = fresh(g1);
      const cx<T>* a2 = fresh(g2);
#pragma unroll
      for (int s = 0; s < kE; ++s) {
        const int i = t + s * TT, k = 2 * i + par;
        u1[par * H + i] = cmulc(v[s], a1[k]);
        u2[par * H + i] = cmulc(v[s], a2[k]);
        issue_fence<true>();   // bound the loads in flight
      }
    }
    // Z = G1 FFT_P(trunc_L IFFT_P(U1)) - G2 FFT_P(trunc_L IFFT_P(U2)), into U1
#pragma unroll 1
    for (int br = 0; br < 2; ++br) {
      cx<T>* const U = br ? U2 : U1;
      const cx<T>* const g = br ? g2 : g1;
      load(U);                                           // a = IFFT_H(even half)
      inv();
      store(U);
      load(U + H);                                       // b = IFFT_H(odd half)
      inv();
      {
        cx<T>* u = fresh(U);
        const cx<T>* tw = fresh(twg);
#pragma unroll
        for (int s = 0; s < kE; ++s) {                   // p = a + W^-n b (n < L) to U;
          const int i = t + s * TT;                      // v = p W^n
          const cx<T> wi = split_twiddle<P>(tw, i);
          const cx<T> pv = (i < L) ? u[i] + cmulc(v[s], wi) : cx<T>{0, 0};
          u[i] = pv;
          v[s] = cmul(pv, wi);
          issue_fence<true>();   // bound the loads in flight
        }
      }
      fwd();                                             // odd half of FFT_P(p)
      {
        cx<T>* z1 = fresh(U1);
        const cx<T>* a = fresh(g);
#pragma unroll
        for (int s = 0; s < kE; ++s) {
          const int i = t + s * TT;
          const cx<T> z = cmul(v[s], a[2 * i + 1]);
          z1[H + i] = br ? z1[H + i] - z : z;
          issue_fence<true>();   // bound the loads in flight
        }
      }
      load(U);                                           // even half of FFT_P(p)
      fwd();
      {
        cx<T>* z1 = fresh(U1);
        const cx<T>* a = fresh(g);
#pragma unroll
        for (int s = 0; s < kE; ++s) {
          const int i = t + s * TT;
          const cx<T> z = cmul(v[s], a[2 * i]);
          z1[i] = br ? z1[i] - z : z;
          issue_fence<true>();   // bound the loads in flight
        }
      }
    }
    // beta = trunc_L IFFT_P(Z); F_u: beams = post3 * IFFT_P(H3 FFT_P(beta * pre3))[0:N]
    load(U1);
    inv();
    store(U1);
    load(U1 + H);
    inv();
    {
      cx<T>* u = fresh(U1);
      const cx<T>* tw = fresh(twg);
      const cx<T>* pre = fresh(pre3);
#pragma unroll
      for (int s = 0; s < kE; ++s) {                     // y = beta pre3 to U1; v = y W^n
        const int i = t + s * TT;
        const cx<T> wi = split_twiddle<P>(tw, i);
        const cx<T> y = (i < L) ? cmul(u[i] + cmulc(v[s], wi), pre[i]) : cx<T>{0, 0};
        u[i] = y;
        v[s] = cmul(y, wi);
        issue_fence<true>();   // bound the loads in flight
      }
    }
    fwd();                                               // odd half of FFT_P(y), times H3,
    {                                                    // then its H-point inverse (b)
      const cx<T>* h = fresh(H3);
#pragma unroll
      for (int s = 0; s < kE; ++s) v[s] = cmul(v[s], h[2 * (t + s * TT) + 1]);
    }
    inv();
    store(U1 + H);
    load(U1);                                            // even half, times H3, inverse (a)
    fwd();
    {
      const cx<T>* h = fresh(H3);
#pragma unroll
      for (int s = 0; s < kE; ++s) v[s] = cmul(v[s], h[2 * (t + s * TT)]);
    }
    inv();
    {
      cx<TOUT>* dst = static_cast<cx<TOUT>*>(outs.p[blk]) + static_cast<size_t>(bm) * N;
      const cx<T>* u = fresh(U1);
      const cx<T>* tw = fresh(twg);
      const cx<T>* post = fresh(post3);
#pragma unroll
      for (int s = 0; s < kE; ++s) {                     // x[n] = a + W^-n b, x[n + H] = a - W^-n b
        const int i = t + s * TT;
        const cx<T> wb = cmulc(u[H + i], split_twiddle<P>(tw, i));
        if (i < N) dst[i] = cvt<TOUT>(cmul(v[s] + wb, post[i]));
        if (i + H < N) dst[i + H] = cvt<TOUT>(cmul(v[s] - wb, post[i + H]));
        issue_fence<true>();   // bound the loads in flight
      }
    }
  }
}

}  // namespace

size_t split_scratch_bytes(int P, bool dbl) {
  return dbl ? static_cast<size_t>(split_grid<double>()) * 2 * P * sizeof(cx<double>)
             : static_cast<size_t>(split_grid<float>()) * 2 * P * sizeof(cx<float>);
}

template <typename T, typename TIN, typename TOUT>
hipError_t launch_toeplitz_fu_split(int P, const void* w, const OutPtrs& outs, const void* G1,
                                    const void* G2, const void* pre3, const void* H3,
                                    const void* post3, const void* tw, void* scratch, int B, int L,
                                    int N, int nblocks, hipStream_t st) {
  if (nblocks < 1 || nblocks > MAX_LAUNCH_BLOCKS || !scratch) return hipErrorInvalidValue;
  if (2 * L > P || N + L - 1 > P) return hipErrorInvalidValue;
  const int grid = std::min(split_grid<T>(), nblocks * B);
  switch (P) {
#define CASE(PP)                                                                               \
  case PP:                                                                                     \
    hipLaunchKernelGGL((k_toeplitz_fu_split<T, TIN, TOUT, PP>), dim3(grid),                    \
                       dim3(Shape<PP / 2>::THREADS), 0, st, (const cx<TIN>*)w, outs,           \
                       (const cx<T>*)G1, (const cx<T>*)G2, (const cx<T>*)pre3,                 \
                       (const cx<T>*)H3, (const cx<T>*)post3, (const cx<T>*)tw,                \
                       B, L, N, nblocks, (cx<T>*)scratch);                                     \
    return hipGetLastError();
    CASE(8192) CASE(16384)
#undef CASE
    default:
      break;
  }
  return hipErrorInvalidValue;
}

#define FBST_SPLIT_INST(T, TIN, TOUT)                                                          \
  template hipError_t launch_toeplitz_fu_split<T, TIN, TOUT>(                                  \
      int, const void*, const OutPtrs&, const void*, const void*, const void*, const void*,    \
      const void*, const void*, void*, int, int, int, int, hipStream_t);
FBST_SPLIT_INST(double, float, float)
FBST_SPLIT_INST(double, double, double)
#undef FBST_SPLIT_INST

template hipError_t launch_toeplitz_fu<float, float, float>(
    int, const void*, const OutPtrs&, const void*, const void*, const void*, const void*, const void*,
    const void*, int, int, int, int, hipStream_t, int);
template hipError_t launch_toeplitz_fu<double, float, float>(
    int, const void*, const OutPtrs&, const void*, const void*, const void*, const void*, const void*,
    const void*, int, int, int, int, hipStream_t, int);
template hipError_t launch_toeplitz_fu<double, double, double>(
    int, const void*, const OutPtrs&, const void*, const void*, const void*, const void*, const void*,
    const void*, int, int, int, int, hipStream_t, int);

}  // namespace fbst
