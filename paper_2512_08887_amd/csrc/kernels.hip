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
//
// Zero padding is declared to the FFTs at compile time (SI = register slots
// that can hold input, SO = register slots whose output is used), so first
// passes skip zero operands and last passes compute only used outputs.
//
// Workgroups are remapped so that each XCD (each L2) receives a contiguous
// range of the logical work: per-frequency tables of K2 and per-beam spectra
// of K3 are then fetched into one L2 and reused there.
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

// ---------------------------------------------------------------------------
// K1: Yhat[row][i] = post[i] * IFFT(FFT(x[row][n] * pre[n]) * H)[i],  i < L.
// rows are (block, sensor) pairs; lane = g * TT + t (a transform owns a
// contiguous run of lanes, so row loads and stores are coalesced).
// SI >= ceil(N / TT), SO >= ceil(L / TT).
// ---------------------------------------------------------------------------
template <typename T, int P, int SI, int SO>
__global__ __launch_bounds__(Shape<P>::THREADS) FBST_K12_ATTR void k_time_czt(
    const InPtrs xs, cx<T>* __restrict__ yhat, const cx<T>* __restrict__ pre,
    const cx<T>* __restrict__ H, const cx<T>* __restrict__ post, const cx<T>* __restrict__ tw,
    int M, int N, int L, int rows) {
  using SH = Shape<P>;
  __shared__ cx<T> lds[SH::G * SH::S];
  const int g = threadIdx.x / SH::TT;
  const int t = threadIdx.x % SH::TT;
  const int row = blockIdx.x * SH::G + g;
  const bool active = row < rows;
  cx<T>* buf = lds + g * SH::S;

  cx<T> v[kE];
  const int rr = active ? row : 0;                    // inactive lanes read row 0, store nothing
  const int blk = rr / M;
  const cx<T>* src = static_cast<const cx<T>*>(xs.p[blk]) + (rr - blk * M) * (xs.ld > 0 ? xs.ld : N);
  // Loads at clamped indices and a select afterwards (no branch per load, so
  // the loads are issued together rather than one round trip each).
  {
    cx<T> xa[SI], pa[SI];
#pragma unroll
    for (int s = 0; s < SI; ++s) {
      const int n = t + s * SH::TT;
      const int nc = n < N ? n : N - 1;
      xa[s] = ldg(src + nc);
      pa[s] = ldg(pre + nc);
    }
    issue_fence();
#pragma unroll
    for (int s = 0; s < SI; ++s) v[s] = (t + s * SH::TT < N) ? cmul(xa[s], pa[s]) : cx<T>{0, 0};
  }
#pragma unroll
  for (int s = SI; s < kE; ++s) v[s] = cx<T>{0, 0};
  fft<T, P, kE, -1, SI, FBST_K12_TW>(v, buf, tw, t);
  {
    cx<T> h[kE];
#pragma unroll
    for (int s = 0; s < kE; ++s) h[s] = ldg(H + t + s * SH::TT);
    issue_fence();
#pragma unroll
    for (int s = 0; s < kE; ++s) v[s] = cmul(v[s], h[s]);
  }
  fft<T, P, kE, +1, kE, FBST_K12_TW>(v, buf, tw, t);
  cx<T>* dst = yhat + static_cast<size_t>(row) * L;
  cx<T> po[SO];
#pragma unroll
  for (int s = 0; s < SO; ++s) {
    const int i = t + s * SH::TT;
    po[s] = ldg(post + (i < L ? i : L - 1));
  }
  issue_fence();
#pragma unroll
  for (int s = 0; s < SO; ++s) {
    const int i = t + s * SH::TT;
    if (active && i < L) dst[i] = cmul(v[s], po[s]);
  }
}

// ---------------------------------------------------------------------------
// K1, split-output form.  The L outputs are two halves of Ls = L/2 each; half
// h needs the chirp kernel only over [-(N-1), Ls-1] shifted by h Ls, so both
// halves are circular convolutions of P >= N + Ls - 1 points (P1 / 2 when
// L = 2N) that share the forward transform of the premultiplied input:
//   X = FFT(x pre);  Yhat[h Ls + i] = post[h Ls + i] IFFT(X Hh)[i],  h = 0, 1,
// three P-point transforms instead of two of 2P (the two inverses run as one
// dual transform).  SI >= ceil(N / TT), SO >= ceil(Ls / TT).
// ---------------------------------------------------------------------------
#ifndef FBST_K1S_DUAL
#define FBST_K1S_DUAL 1           // run the two inverse transforms as one dual transform
#endif
constexpr int kK1sBufs = FBST_K1S_DUAL ? 2 : 1;
#ifndef FBST_K1S_WAVES
#define FBST_K1S_WAVES 0          // minimum waves per SIMD for the split stage 1a (0: compiler's choice)
#endif
#if FBST_K1S_WAVES > 0
#define FBST_K1S_ATTR __attribute__((amdgpu_waves_per_eu(FBST_K1S_WAVES)))
#else
#define FBST_K1S_ATTR
#endif

template <typename T, int P>
constexpr bool k1s_fits() {
  return sizeof(T) * 2 * lds_stride(P) * kK1sBufs * Shape<P>::G <= 160 * 1024;
}

template <typename T, int P, int SI, int SO>
__global__ __launch_bounds__(Shape<P>::THREADS) FBST_K1S_ATTR void k_time_czt_split(
    const InPtrs xs, cx<T>* __restrict__ yhat, const cx<T>* __restrict__ pre,
    const cx<T>* __restrict__ Ha, const cx<T>* __restrict__ Hb, const cx<T>* __restrict__ post,
    const cx<T>* __restrict__ tw, int M, int N, int L, int Ls, int rows) {
  using SH = Shape<P>;
  __shared__ cx<T> lds[SH::G * kK1sBufs * SH::S];
  const int g = threadIdx.x / SH::TT;
  const int t = threadIdx.x % SH::TT;
  const int row = blockIdx.x * SH::G + g;
  const bool active = row < rows;
  cx<T>* buf = lds + g * kK1sBufs * SH::S;

  cx<T> v[kE], u[kE];
  const int rr = active ? row : 0;                    // inactive lanes read row 0, store nothing
  const int blk = rr / M;
  const cx<T>* src = static_cast<const cx<T>*>(xs.p[blk]) + (rr - blk * M) * (xs.ld > 0 ? xs.ld : N);
  {
    cx<T> xa[SI], pa[SI];
#pragma unroll
    for (int s = 0; s < SI; ++s) {
      const int n = t + s * SH::TT;
      const int nc = n < N ? n : N - 1;
      xa[s] = ldg(src + nc);
      pa[s] = ldg(pre + nc);
    }
    issue_fence();
#pragma unroll
    for (int s = 0; s < SI; ++s) v[s] = (t + s * SH::TT < N) ? cmul(xa[s], pa[s]) : cx<T>{0, 0};
  }
#pragma unroll
  for (int s = SI; s < kE; ++s) v[s] = cx<T>{0, 0};
  fft<T, P, kE, -1, SI, FBST_K12_TW>(v, buf, tw, t);
  {
    cx<T> ha[kE], hb[kE];
#pragma unroll
    for (int s = 0; s < kE; ++s) {
      ha[s] = ldg(Ha + t + s * SH::TT);
      hb[s] = ldg(Hb + t + s * SH::TT);
    }
    issue_fence();
#pragma unroll
    for (int s = 0; s < kE; ++s) {
      u[s] = cmul(v[s], hb[s]);
      v[s] = cmul(v[s], ha[s]);
    }
  }
  if constexpr (FBST_K1S_DUAL) {
    fft2<T, P, kE, +1, kE, FBST_K12_TW>(v, u, buf, buf + SH::S, tw, t);
  } else {
    fft<T, P, kE, +1, kE, FBST_K12_TW>(v, buf, tw, t);
    fft<T, P, kE, +1, kE, FBST_K12_TW>(u, buf, tw, t);
  }
  cx<T>* dst = yhat + static_cast<size_t>(row) * L;
  cx<T> pa[SO], pb[SO];
#pragma unroll
  for (int s = 0; s < SO; ++s) {
    const int i = t + s * SH::TT;
    pa[s] = ldg(post + (i < Ls ? i : Ls - 1));
    pb[s] = ldg(post + (i < L - Ls ? Ls + i : L - 1));
  }
  issue_fence();
#pragma unroll
  for (int s = 0; s < SO; ++s) {
    const int i = t + s * SH::TT;
    if (active && i < Ls) dst[i] = cmul(v[s], pa[s]);
    if (active && i < L - Ls) dst[Ls + i] = cmul(u[s], pb[s]);
  }
}

// ---------------------------------------------------------------------------
// K2: one axis of the space chirp-z.  Data layout [blk][pre_n][A][post_n][L]
// (A = a_in on input, a_out on output); a workgroup takes G consecutive l for
// one (blk, p, q) and lane = t * G + g, so lanes with the same t read G
// consecutive l of one element.  Tables are l-fastest: pre [a_in][L],
// H [P][L], post [a_out][L].  Logical work order: l-tile outermost, so the
// workgroups of one XCD share the tables of a few tiles.
// SI >= ceil(a_in / TT), SO >= ceil(a_out / TT).
// ---------------------------------------------------------------------------
template <typename T, int P, int SI, int SO>
__global__ __launch_bounds__(ShapeK2<P>::THREADS) FBST_K12_ATTR void k_axis_czt(
    const cx<T>* __restrict__ in, cx<T>* __restrict__ out, const cx<T>* __restrict__ pre,
    const cx<T>* __restrict__ H, const cx<T>* __restrict__ post, const cx<T>* __restrict__ tw,
    int a_in, int a_out, int pre_n, int post_n, int L, int nblocks, int n_tiles) {
  using SH = ShapeK2<P>;
  __shared__ cx<T> lds[SH::G * SH::S];
  const int g = threadIdx.x % SH::G;
  const int t = threadIdx.x / SH::G;
  int w = xcd_linear(gridDim.x);
  const int q = w % post_n;
  w /= post_n;
  const int p = w % pre_n;
  w /= pre_n;
  const int blk = w % nblocks;
  const int tile = w / nblocks;
  const int l = tile * SH::G + g;
  const bool active = l < L;
  cx<T>* buf = lds + g * SH::S;

  const int lc = active ? l : L - 1;                  // inactive lanes read a valid l, store nothing
  const size_t stride = static_cast<size_t>(post_n) * L;
  const cx<T>* src = in + ((static_cast<size_t>(blk) * pre_n + p) * a_in * post_n + q) * L + lc;
  cx<T> v[kE];
  {
    cx<T> xa[SI], pa[SI];
#pragma unroll
    for (int s = 0; s < SI; ++s) {
      const int i = t + s * SH::TT;
      const int ic = i < a_in ? i : a_in - 1;
      xa[s] = ldg(src + ic * stride);
      pa[s] = ldg(pre + static_cast<size_t>(ic) * L + lc);
    }
    issue_fence();
#pragma unroll
    for (int s = 0; s < SI; ++s)
      v[s] = (active && t + s * SH::TT < a_in) ? cmul(xa[s], pa[s]) : cx<T>{0, 0};
  }
#pragma unroll
  for (int s = SI; s < kE; ++s) v[s] = cx<T>{0, 0};
  fft<T, P, kE, -1, SI, FBST_K12_TW>(v, buf, tw, t);
  {
    cx<T> h[kE];
#pragma unroll
    for (int s = 0; s < kE; ++s) h[s] = ldg(H + static_cast<size_t>(t + s * SH::TT) * L + lc);
    issue_fence();
#pragma unroll
    for (int s = 0; s < kE; ++s) v[s] = cmul(v[s], h[s]);
  }
  fft<T, P, kE, +1, kE, FBST_K12_TW>(v, buf, tw, t);
  cx<T>* dst = out + ((static_cast<size_t>(blk) * pre_n + p) * a_out * post_n + q) * L + l;
  cx<T> po[SO];
#pragma unroll
  for (int s = 0; s < SO; ++s) {
    const int a = t + s * SH::TT;
    po[s] = ldg(post + static_cast<size_t>(a < a_out ? a : a_out - 1) * L + lc);
  }
  issue_fence();
#pragma unroll
  for (int s = 0; s < SO; ++s) {
    const int a = t + s * SH::TT;
    if (active && a < a_out) dst[a * stride] = cmul(v[s], po[s]);
  }
}

// ---------------------------------------------------------------------------
// Stage 1b for arbitrary element positions (Sec. IX, eq. DFT_non_unif): per
// frequency l a type-1 non-uniform FFT over the modes of the beam grid.
//   spread: c_m = Yhat[m][l] pre[m][l] is spread onto an oversampled grid
//     (nfx x nfy cells per frequency, in LDS) with a W-point exponential-of-
//     semicircle kernel per axis, and the grid is written out as
//     [blk][nfx][nfy][L];
//   k_axis_dft: per axis, an nf-point FFT (exp(+j)) of the grid and the output
//     modes a - a_out/2, each scaled by the deconvolution factor corr[a].
// The spread needs no atomics: every cell update is a read and a write of LDS
// by the one lane that owns it at that moment, and a wave's LDS operations
// complete in program order, so the grid is the same bit for bit on every run.
// ---------------------------------------------------------------------------

// Kernel value of tap t (grid cell j0 + t) for a point f cells beyond cell
// j0 + W/2 - 1: phi(z), z = (t - W/2 + 1 - f) 2 / W,
// phi(z) = exp(beta (sqrt(1 - z^2) - 1)) = 2^(b2 sqrt(1 - z^2) - b2) with
// b2 = beta log2(e) (the caller passes b2).  float: the hardware square root
// and base-2 exponential (about 1 ulp each, far below the kernel's own
// accuracy); double: the library functions.
template <typename T, int W>
__device__ __forceinline__ T es_tap(int t, T f, T b2) {
  constexpr T s = static_cast<T>(2.0 / W);
  const T z = static_cast<T>(t - W / 2 + 1) * s - f * s;
  const T q = static_cast<T>(1) - z * z;
  const T qc = q > static_cast<T>(0) ? q : static_cast<T>(0);
  if constexpr (sizeof(T) == 4) return __builtin_amdgcn_exp2f(b2 * __builtin_amdgcn_sqrtf(qc) - b2);
  else return ::exp2(b2 * ::sqrt(qc) - b2);
}

// LDS layout of the grids.  Line: cell c at word c + c / 16 (one pad word per
// 16 cells, so cells 16, 32 or 64 apart -- the spacing of elements spread at
// once -- fall in different banks).  Plane: cell (jx, jy) at word
// jx (nfy + 8) + jy, so the W x W taps of one element spread over the banks.
// Consecutive frequencies' grids start 8 banks apart (stride = 8 mod 32).
__device__ __forceinline__ int swz(int c) { return c + (c >> 4); }
__host__ __device__ constexpr int spread_words(int nfx, int nfy) {
  return nfy > 1 ? nfx * (nfy + 8) : nfx + nfx / 16;
}
__host__ __device__ constexpr int spread_stride(int nfx, int nfy) {
  return spread_words(nfx, nfy) + ((40 - spread_words(nfx, nfy) % 32) % 32);
}

// Zero the G padded grids, or write them out to [blk][cells][L] at l = l0 + g.
template <typename T>
__device__ __forceinline__ void spread_zero(T* lds, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) lds[i] = static_cast<T>(0);
}
template <typename T, typename Word>
__device__ __forceinline__ void spread_store(const T* re, const T* im, int S, int cells, int G,
                                             cx<T>* dst, int l0, int L, Word&& word) {
  for (int i = threadIdx.x; i < cells * G; i += blockDim.x) {
    const int g = i % G, j = i / G;
    if (l0 + g < L) dst[static_cast<size_t>(j) * L + g] = cx<T>{re[g * S + word(j)], im[g * S + word(j)]};
  }
}

constexpr int kSpreadGroup = 8;               // elements whose loads are in flight together

// Line of beams (nfy = 1).  A workgroup takes G consecutive frequencies of one
// block with R lanes each (lane = r Gw + g' inside a wave of Gw frequencies,
// so the Gw lanes of one r read Gw consecutive l).  Lane r takes the elements
// order[r C + s], s < C = ceil(M / R), in turn: W cells read, updated, written.
// The plan chooses R such that the supports of the R elements of one step are
// disjoint at every frequency, so no cell is touched by two lanes at once.
// Element data are loaded a group ahead (row indices two groups ahead).
struct LineLane {
  int g, r;        // frequency within the workgroup, lane within the frequency
};
__device__ __forceinline__ LineLane line_lane(int G, int R) {
  const int Gw = (G * R > 64) ? 64 / R : G;
  const int i = threadIdx.x, per_wave = Gw * R;
  return {(i / per_wave) * Gw + i % Gw, (i % per_wave) / Gw};
}

// Lane r's run of elements spread into the grid (gre, gim) of frequency l.
template <typename T, int W>
__device__ __forceinline__ void spread_line_run(const cx<T>* __restrict__ src,
                                                const cx<T>* __restrict__ pre,
                                                const cx<T>* __restrict__ pos,
                                                const int* __restrict__ order, int k0, int k1,
                                                int nf, int l, int L, T b2, T* gre, T* gim) {
  constexpr int D = kSpreadGroup;
  auto rows = [&](int base, int (&mm)[D]) {
#pragma unroll
    for (int d = 0; d < D; ++d) mm[d] = order[base + d < k1 ? base + d : k0];
  };
  auto fetch = [&](const int (&mm)[D], cx<T> (&y)[D], cx<T> (&pr)[D], cx<T> (&ps)[D]) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const size_t idx = static_cast<size_t>(mm[d]) * L;
      y[d] = ldg(src + idx);
      pr[d] = ldg(pre + idx + l);
      ps[d] = ldg(pos + idx + l);
    }
  };
  int mm[D], mn[D];
  cx<T> y[D], pr[D], ps[D];
  rows(k0, mm);
  fetch(mm, y, pr, ps);
  rows(k0 + D, mn);
  for (int base = k0; base < k1; base += D) {
    cx<T> y2[D], pr2[D], ps2[D];
    const bool more = base + D < k1;
    if (more) {
      fetch(mn, y2, pr2, ps2);
      rows(base + 2 * D, mn);
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if (base + d < k1) {
        const cx<T> c = cmul(y[d], pr[d]);
        const T f = ps[d].re;
        const int j0 = static_cast<int>(ps[d].im);
        int cell[W];
        T ar[W], ai[W];
#pragma unroll
        for (int t = 0; t < W; ++t) {
          cell[t] = swz((j0 + t) & (nf - 1));
          ar[t] = gre[cell[t]];
          ai[t] = gim[cell[t]];
        }
#pragma unroll
        for (int t = 0; t < W; ++t) {
          const T kv = es_tap<T, W>(t, f, b2);
          gre[cell[t]] = ar[t] + c.re * kv;
          gim[cell[t]] = ai[t] + c.im * kv;
        }
      }
    }
    if (more) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        y[d] = y2[d];
        pr[d] = pr2[d];
        ps[d] = ps2[d];
      }
    }
  }
}

template <typename T, int W, int LDS_BYTES>
__global__ __launch_bounds__(256) void k_nu_spread_line(
    const cx<T>* __restrict__ in, cx<T>* __restrict__ out, const cx<T>* __restrict__ pre,
    const cx<T>* __restrict__ pos, const int* __restrict__ order, int M, int nf, int G, int R,
    T b2, int L, int nblocks) {
  __shared__ T grid_lds[LDS_BYTES / sizeof(T)];
  const int S = spread_stride(nf, 1);
  T* re = grid_lds;
  T* im = grid_lds + S * G;
  const int wl = xcd_linear(gridDim.x);
  const int blk = wl % nblocks;
  const int tile = wl / nblocks;
  const LineLane ln = line_lane(G, R);
  spread_zero(grid_lds, 2 * S * G);
  __syncthreads();
  const int l = tile * G + ln.g;
  const int C = (M + R - 1) / R;
  const int k0 = ln.r * C, k1 = min(M, k0 + C);
  if (l < L && k0 < k1)
    spread_line_run<T, W>(in + static_cast<size_t>(blk) * M * L + l, pre, pos, order, k0, k1, nf,
                          l, L, b2, re + ln.g * S, im + ln.g * S);
  __syncthreads();
  spread_store(re, im, S, nf, G, out + static_cast<size_t>(blk) * nf * L + static_cast<size_t>(tile) * G,
               tile * G, L, [](int j) { return swz(j); });
}

// Line of beams, fused: the spread as above into per-frequency regions of 2 Sf
// words (re at 0, im at Sf), then in rounds of NT = 256 / TT frequencies the
// P-point FFT (exp(+j)) of each grid, its scratch laid over the grid's own
// region once the grid is in registers, and the modes a - a_out/2 scaled by
// corr[a] stored to w [blk][a][l]: the oversampled grid never leaves LDS.
// FFT lanes: lane = t NT + g' (the NT lanes of one t store NT consecutive l).
__host__ __device__ constexpr int fused_stride(int P) {
  return P + P / 16 + (((4 - (P + P / 16) % 32) + 32) % 32 == 0 ? 32 : ((4 - (P + P / 16) % 32) + 32) % 32);
}

template <typename T, int W, int P, int LDS_BYTES>
__global__ __launch_bounds__(256) void k_nu_line_fused(
    const cx<T>* __restrict__ in, cx<T>* __restrict__ wout, const cx<T>* __restrict__ pre,
    const cx<T>* __restrict__ pos, const int* __restrict__ order, const cx<T>* __restrict__ corr,
    const cx<T>* __restrict__ tw, int M, int G, int R, T b2, int L, int nblocks, int a_out) {
  constexpr int TT = P / kE, NT = 256 / TT;
  constexpr int Sf = fused_stride(P);
  static_assert(Sf >= lds_stride(P), "a grid region must hold the FFT scratch");
  __shared__ alignas(16) T grid_lds[LDS_BYTES / sizeof(T)];
  const int wl = xcd_linear(gridDim.x);
  const int blk = wl % nblocks;
  const int tile = wl / nblocks;
  spread_zero(grid_lds, 2 * Sf * G);
  __syncthreads();
  {
    const LineLane ln = line_lane(G, R);
    const int l = tile * G + ln.g;
    const int C = (M + R - 1) / R;
    const int k0 = ln.r * C, k1 = min(M, k0 + C);
    if (threadIdx.x < G * R && l < L && k0 < k1)
      spread_line_run<T, W>(in + static_cast<size_t>(blk) * M * L + l, pre, pos, order, k0, k1, P,
                            l, L, b2, grid_lds + 2 * Sf * ln.g, grid_lds + 2 * Sf * ln.g + Sf);
  }
  __syncthreads();
  const int gi = threadIdx.x % NT, t = threadIdx.x / NT, ka = a_out / 2;
  for (int g0 = 0; g0 < G; g0 += NT) {
    const int g = g0 + gi, l = tile * G + g;
    const T* gre = grid_lds + 2 * Sf * g;
    cx<T> v[kE];
#pragma unroll
    for (int s = 0; s < kE; ++s) {
      const int c = swz(t + s * TT);
      v[s] = cx<T>{gre[c], gre[Sf + c]};
    }
    // the FFT's first write to its scratch follows a workgroup barrier, after
    // which every lane holds its grid values in registers
    fft<T, P, kE, +1, kE, FBST_K12_TW>(v, reinterpret_cast<cx<T>*>(grid_lds + 2 * Sf * g), tw, t);
    T cs[kE];
#pragma unroll
    for (int s = 0; s < kE; ++s) {
      const int a = (t + s * TT + ka) & (P - 1);
      cs[s] = ldg(corr + (a < a_out ? a : 0)).re;
    }
    cx<T>* dst = wout + static_cast<size_t>(blk) * a_out * L + l;
#pragma unroll
    for (int s = 0; s < kE; ++s) {
      const int a = (t + s * TT + ka) & (P - 1);
      if (l < L && a < a_out) dst[static_cast<size_t>(a) * L] = cx<T>{v[s].re * cs[s], v[s].im * cs[s]};
    }
  }
}

// 2-D beam grid.  One wave per frequency (G waves); lane q takes the taps
// q + 64 i, i < TPL, as (tx, ty) = (tap / W, tap % W), of every element in
// turn: the W x W cells of one element are distinct, so each cell update of a
// step has one owner.  Element data are loaded a group ahead.
template <typename T, int W>
__device__ __forceinline__ void spread_plane_run(const cx<T>* __restrict__ src,
                                                 const cx<T>* __restrict__ pre,
                                                 const cx<T>* __restrict__ posx,
                                                 const cx<T>* __restrict__ posy, int M, int nfx,
                                                 int nfy, int row, int l, int L, T b2, T* gre,
                                                 T* gim) {
  constexpr int TPL = (W * W + 63) / 64;
  constexpr int D = kSpreadGroup;
  static_assert(TPL * 64 == W * W, "W * W must be a multiple of 64");
  const int q = threadIdx.x % 64;
  auto fetch = [&](int base, cx<T> (&y)[D], cx<T> (&pr)[D], cx<T> (&px)[D], cx<T> (&py)[D]) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const size_t idx = static_cast<size_t>(base + d < M ? base + d : 0) * L;
      y[d] = ldg(src + idx);
      pr[d] = ldg(pre + idx + l);
      px[d] = ldg(posx + idx + l);
      py[d] = ldg(posy + idx + l);
    }
  };
  cx<T> y[D], pr[D], px[D], py[D];
  fetch(0, y, pr, px, py);
  for (int base = 0; base < M; base += D) {
    cx<T> y2[D], pr2[D], px2[D], py2[D];
    const bool more = base + D < M;
    if (more) fetch(base + D, y2, pr2, px2, py2);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if (base + d < M) {
        const cx<T> c = cmul(y[d], pr[d]);
        const int jx0 = static_cast<int>(px[d].im), jy0 = static_cast<int>(py[d].im);
        int cell[TPL];
        T ar[TPL], ai[TPL];
#pragma unroll
        for (int u = 0; u < TPL; ++u) {
          const int tap = q + 64 * u, tx = tap / W, ty = tap % W;
          cell[u] = ((jx0 + tx) & (nfx - 1)) * row + ((jy0 + ty) & (nfy - 1));
          ar[u] = gre[cell[u]];
          ai[u] = gim[cell[u]];
        }
#pragma unroll
        for (int u = 0; u < TPL; ++u) {
          const int tap = q + 64 * u, tx = tap / W, ty = tap % W;
          const T kv = es_tap<T, W>(tx, px[d].re, b2) * es_tap<T, W>(ty, py[d].re, b2);
          gre[cell[u]] = ar[u] + c.re * kv;
          gim[cell[u]] = ai[u] + c.im * kv;
        }
      }
    }
    if (more) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        y[d] = y2[d];
        pr[d] = pr2[d];
        px[d] = px2[d];
        py[d] = py2[d];
      }
    }
  }
}

template <typename T, int W, int LDS_BYTES>
__global__ __launch_bounds__(256) void k_nu_spread_plane(
    const cx<T>* __restrict__ in, cx<T>* __restrict__ out, const cx<T>* __restrict__ pre,
    const cx<T>* __restrict__ posx, const cx<T>* __restrict__ posy, int M, int nfx, int nfy, int G,
    T b2, int L, int nblocks) {
  __shared__ T grid_lds[LDS_BYTES / sizeof(T)];
  const int cells = nfx * nfy, S = spread_stride(nfx, nfy), row = nfy + 8;
  T* re = grid_lds;
  T* im = grid_lds + S * G;
  const int wl = xcd_linear(gridDim.x);
  const int blk = wl % nblocks;
  const int tile = wl / nblocks;
  const int g = threadIdx.x / 64;
  spread_zero(grid_lds, 2 * S * G);
  __syncthreads();
  const int l = tile * G + g;
  if (l < L)
    spread_plane_run<T, W>(in + static_cast<size_t>(blk) * M * L + l, pre, posx, posy, M, nfx, nfy,
                           row, l, L, b2, re + g * S, im + g * S);
  __syncthreads();
  spread_store(re, im, S, cells, G,
               out + static_cast<size_t>(blk) * cells * L + static_cast<size_t>(tile) * G, tile * G, L,
               [nfy, row](int j) { return (j / nfy) * row + j % nfy; });
}

// 2-D beam grid on a 32 x 32 oversampled grid, fused: the spread as above
// into per-frequency regions of 2 S32 words (re at 0, im at S32, rows of 40
// words), then per frequency (one wave) the 32 row FFTs and the 32 column FFTs
// (exp(+j); 2 lanes per transform, the scratch laid over the region once the
// grid is in registers) and the modes (a - bu/2, c - bv/2) scaled by
// cx[a] cy[c] stored to w [blk][a bv + c][l]: the grid never leaves LDS.
constexpr int kPlaneRow = 40;
constexpr int kPlaneS = 32 * kPlaneRow + 8;

template <typename T, int W, int LDS_BYTES>
__global__ __launch_bounds__(256) void k_nu_plane_fused(
    const cx<T>* __restrict__ in, cx<T>* __restrict__ wout, const cx<T>* __restrict__ pre,
    const cx<T>* __restrict__ posx, const cx<T>* __restrict__ posy, const cx<T>* __restrict__ cxs,
    const cx<T>* __restrict__ cys, const cx<T>* __restrict__ tw, int M, int G, int bu, int bv,
    T b2, int L, int nblocks) {
  constexpr int P = 32, TT = P / kE;                 // 2 lanes per 32-point transform
  static_assert(32 * lds_stride(P) <= kPlaneS, "a region must hold 32 transforms' scratch");
  __shared__ alignas(16) T grid_lds[LDS_BYTES / sizeof(T)];
  const int wl = xcd_linear(gridDim.x);
  const int blk = wl % nblocks;
  const int tile = wl / nblocks;
  const int g = threadIdx.x / 64, q = threadIdx.x % 64;
  const int l = tile * G + g;
  T* gre = grid_lds + 2 * kPlaneS * g;
  T* gim = gre + kPlaneS;
  cx<T>* scratch = reinterpret_cast<cx<T>*>(gre);
  spread_zero(grid_lds, 2 * kPlaneS * G);
  __syncthreads();
  if (l < L)
    spread_plane_run<T, W>(in + static_cast<size_t>(blk) * M * L + l, pre, posx, posy, M, P, P,
                           kPlaneRow, l, L, b2, gre, gim);
  __syncthreads();
  const int r = q / TT, t = q % TT;                  // transform (row, then column) and its lane
  cx<T> v[kE];
  // rows: v[s] = cell (r, t + TT s)
#pragma unroll
  for (int s = 0; s < kE; ++s) {
    const int c = r * kPlaneRow + t + TT * s;
    v[s] = cx<T>{gre[c], gim[c]};
  }
  fft<T, P, kE, +1, kE, FBST_K12_TW>(v, scratch + r * lds_stride(P), tw, t);
  __syncthreads();                                   // every lane is done with the scratch
#pragma unroll
  for (int s = 0; s < kE; ++s) {
    const int c = r * kPlaneRow + t + TT * s;
    gre[c] = v[s].re;
    gim[c] = v[s].im;
  }
  __syncthreads();
  // columns: v[s] = cell (t + TT s, r)
#pragma unroll
  for (int s = 0; s < kE; ++s) {
    const int c = (t + TT * s) * kPlaneRow + r;
    v[s] = cx<T>{gre[c], gim[c]};
  }
  fft<T, P, kE, +1, kE, FBST_K12_TW>(v, scratch + r * lds_stride(P), tw, t);
  // v[s] is the spectrum at (kx, ky) = (t + TT s, r)
  const int cy_i = (r + bv / 2) & (P - 1);
  if (l < L && cy_i < bv) {
    const T sy = ldg(cys + cy_i).re;
    cx<T>* dst = wout + static_cast<size_t>(blk) * bu * bv * L + l;
#pragma unroll
    for (int s = 0; s < kE; ++s) {
      const int a = (t + TT * s + bu / 2) & (P - 1);
      if (a < bu) {
        const T sc = ldg(cxs + a).re * sy;
        dst[(static_cast<size_t>(a) * bv + cy_i) * L] = cx<T>{v[s].re * sc, v[s].im * sc};
      }
    }
  }
}

// One axis of the non-uniform stage 1b: layout [blk][pre_n][P][post_n][L] in,
// [blk][pre_n][a_out][post_n][L] out; lane mapping and work order as K2.
// out[a] = corr[a].re * sum_j in[j] exp(+j 2 pi (a - a_out/2) j / P).
template <typename T, int P>
__global__ __launch_bounds__(ShapeK2<P>::THREADS) FBST_K12_ATTR void k_axis_dft(
    const cx<T>* __restrict__ in, cx<T>* __restrict__ out, const cx<T>* __restrict__ corr,
    const cx<T>* __restrict__ tw, int a_out, int pre_n, int post_n, int L, int nblocks) {
  using SH = ShapeK2<P>;
  __shared__ cx<T> lds[SH::G * SH::S];
  const int g = threadIdx.x % SH::G;
  const int t = threadIdx.x / SH::G;
  int w = xcd_linear(gridDim.x);
  const int q = w % post_n;
  w /= post_n;
  const int p = w % pre_n;
  w /= pre_n;
  const int blk = w % nblocks;
  const int tile = w / nblocks;
  const int l = tile * SH::G + g;
  const bool active = l < L;
  cx<T>* buf = lds + g * SH::S;
  const int lc = active ? l : L - 1;
  const size_t stride = static_cast<size_t>(post_n) * L;
  const cx<T>* src = in + ((static_cast<size_t>(blk) * pre_n + p) * P * post_n + q) * L + lc;
  cx<T> v[kE];
#pragma unroll
  for (int s = 0; s < kE; ++s) v[s] = ldg(src + (t + s * SH::TT) * stride);
  issue_fence();
  fft<T, P, kE, +1, kE, FBST_K12_TW>(v, buf, tw, t);
  const int ka = a_out / 2;
  cx<T>* dst = out + ((static_cast<size_t>(blk) * pre_n + p) * a_out * post_n + q) * L + l;
  T cs[kE];
#pragma unroll
  for (int s = 0; s < kE; ++s) {
    const int a = (t + s * SH::TT + ka) & (P - 1);
    cs[s] = ldg(corr + (a < a_out ? a : 0)).re;
  }
  issue_fence();
#pragma unroll
  for (int s = 0; s < kE; ++s) {
    const int a = (t + s * SH::TT + ka) & (P - 1);
    if (active && a < a_out) dst[a * stride] = cx<T>{v[s].re * cs[s], v[s].im * cs[s]};
  }
}

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
constexpr bool k3_dual() {
  return FBST_K3_DUAL && sizeof(T) * 2 * lds_stride(P) * 2 * Shape<P>::G <= 160 * 1024;
}

// Stage 2 with one step of iterative refinement (MODE 1 then MODE 2, two
// launches): the float32 Gohberg-Semencul apply loses accuracy where its two
// terms, each much larger than beta, cancel; a second apply to the residual
// r = w - A beta_1 (A by circulant embedding of its first column, CA =
// FFT(c_0 .. c_{L-1}, 0 .., conj c_{L-1} .. conj c_1) / P) recovers it:
//   MODE 0  beta = GS(w); beams = F_u beta                       (8 transforms)
//   MODE 1  beta_1 = GS(w) stored to bt [rows][L]                (6 transforms)
//   MODE 2  r = w - A beta_1; beta = beta_1 + GS(r); beams = F_u beta (10 transforms)
template <typename T, typename TIN, typename TOUT, int P, int SN, int MODE = 0>
__global__ __launch_bounds__(Shape<P>::THREADS) FBST_K3_ATTR void k_toeplitz_fu(
    const cx<TIN>* __restrict__ w, const OutPtrs outs, const cx<T>* __restrict__ G1,
    const cx<T>* __restrict__ G2, const cx<T>* __restrict__ pre3, const cx<T>* __restrict__ H3,
    const cx<T>* __restrict__ post3, const cx<T>* __restrict__ tw, int B, int L, int N,
    int nblocks, cx<T>* __restrict__ bt = nullptr, const cx<T>* __restrict__ CA = nullptr) {
  using SH = Shape<P>;
  constexpr int SL = kE / 2;
  constexpr bool DUAL = k3_dual<T, P>();
  constexpr int NBUF = DUAL ? 2 : 1;
  __shared__ cx<T> lds[SH::G * NBUF * SH::S];
  const int g = threadIdx.x / SH::TT;
  const int t = threadIdx.x % SH::TT;
  const int rows = nblocks * B;
  const int lw = xcd_linear(gridDim.x) * SH::G + g;     // beam-major logical row
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
    fft<T, P, kE, -1, SL, FBST_K3_TW>(u1, buf, tw, t);
    with_tables<FBST_K3_GB, kE, SH::TT>(CA + static_cast<size_t>(b) * P + t,
                                        static_cast<const cx<T>*>(nullptr),
                                        [&](int s, cx<T> a, cx<T>) { u1[s] = cmul(u1[s], a); });
    fft<T, P, kE, +1, kE, FBST_K3_TW>(u1, buf, tw, t);
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
  fft<T, P, kE, -1, SL, FBST_K3_TW>(u1, buf, tw, t);
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
    fft<T, P, kE, +1, kE, FBST_K3_TW>(u1, buf, tw, t);
#pragma unroll
    for (int s = 0; s < kE; ++s)
      if (s >= SL || t + s * SH::TT >= L) u1[s] = cx<T>{0, 0};
    fft<T, P, kE, -1, SL, FBST_K3_TW>(u1, buf, tw, t);
#pragma unroll
    for (int s = 0; s < kE; ++s) u1[s] = cmul(u1[s], ldg(g1 + t + s * SH::TT));
    // branch 2: u1 -= G2 * FFT(trunc_L(IFFT(u2)))
    fft<T, P, kE, +1, kE, FBST_K3_TW>(u2, buf, tw, t);
#pragma unroll
    for (int s = 0; s < kE; ++s)
      if (s >= SL || t + s * SH::TT >= L) u2[s] = cx<T>{0, 0};
    fft<T, P, kE, -1, SL, FBST_K3_TW>(u2, buf, tw, t);
#pragma unroll
    for (int s = 0; s < kE; ++s) u1[s] = u1[s] - cmul(u2[s], ldg(g2 + t + s * SH::TT));
  }
  // beta = trunc_L(IFFT(Z)), then the F_u chirp-z
  fft<T, P, kE, +1, kE, FBST_K3_TW>(u1, buf, tw, t);
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
  fft<T, P, kE, -1, SL, FBST_K3_TW>(u1, buf, tw, t);
  with_tables<FBST_K3_GB, kE, SH::TT>(H3 + t, static_cast<const cx<T>*>(nullptr),
                                      [&](int s, cx<T> a, cx<T>) { u1[s] = cmul(u1[s], a); });
  fft<T, P, kE, +1, kE, FBST_K3_TW>(u1, buf, tw, t);
  cx<TOUT>* dst = static_cast<cx<TOUT>*>(outs.p[blk]) + static_cast<size_t>(b) * N;
#pragma unroll
  for (int s = 0; s < SN; ++s) {
    const int n = t + s * SH::TT;
    if (active && n < N) dst[n] = cvt<TOUT>(cmul(u1[s], ldg(post3 + n)));
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

}  // namespace

// ---------------------------------------------------------------------------
// Launchers: dispatch the runtime FFT size and slot counts to compiled instances.
// ---------------------------------------------------------------------------
#define FBST_FOR_EACH_P(X) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(8192) X(16384)

template <typename T>
hipError_t launch_time_czt(int P, const InPtrs& xs, int nblocks, void* yhat, const void* pre,
                           const void* H, const void* post, const void* tw, int M, int N, int L,
                           hipStream_t st) {
  if (nblocks < 1 || nblocks > MAX_LAUNCH_BLOCKS) return hipErrorInvalidValue;
  const int rows = nblocks * M;
  switch (P) {
#define CASE(PP)                                                                               \
  case PP:                                                                                     \
    if constexpr (fits_lds<T, PP>()) {                                                         \
      const int si = slots_for<PP>(N), so = slots_for<PP>(L);                                  \
      const dim3 grid(grid_for<PP>(rows)), block(Shape<PP>::THREADS);                          \
      const auto& a = xs;                                                                      \
      const auto o = (cx<T>*)yhat;                                                             \
      if (si <= kE / 4 && so <= kE / 2)                                                        \
        hipLaunchKernelGGL((k_time_czt<T, PP, kE / 4, kE / 2>), grid, block, 0, st, a, o,      \
                           (const cx<T>*)pre, (const cx<T>*)H, (const cx<T>*)post,             \
                           (const cx<T>*)tw, M, N, L, rows);                                   \
      else if (si <= kE / 2)                                                                   \
        hipLaunchKernelGGL((k_time_czt<T, PP, kE / 2, kE>), grid, block, 0, st, a, o,          \
                           (const cx<T>*)pre, (const cx<T>*)H, (const cx<T>*)post,             \
                           (const cx<T>*)tw, M, N, L, rows);                                   \
      else                                                                                     \
        hipLaunchKernelGGL((k_time_czt<T, PP, kE, kE>), grid, block, 0, st, a, o,              \
                           (const cx<T>*)pre, (const cx<T>*)H, (const cx<T>*)post,             \
                           (const cx<T>*)tw, M, N, L, rows);                                   \
      return hipGetLastError();                                                                \
    }                                                                                          \
    break;
    FBST_FOR_EACH_P(CASE)
#undef CASE
    default:
      break;
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_time_czt_split(int P, const InPtrs& xs, int nblocks, void* yhat, const void* pre,
                                 const void* Ha, const void* Hb, const void* post, const void* tw,
                                 int M, int N, int L, int Ls, hipStream_t st) {
  if (nblocks < 1 || nblocks > MAX_LAUNCH_BLOCKS) return hipErrorInvalidValue;
  if (Ls < 1 || Ls > L || L - Ls > Ls || N + Ls - 1 > P) return hipErrorInvalidValue;
  const int rows = nblocks * M;
  switch (P) {
#define CASE(PP)                                                                               \
  case PP:                                                                                     \
    if constexpr (k1s_fits<T, PP>()) {                                                         \
      const int si = slots_for<PP>(N), so = slots_for<PP>(Ls);                                 \
      const dim3 grid(grid_for<PP>(rows)), block(Shape<PP>::THREADS);                          \
      const auto o = (cx<T>*)yhat;                                                             \
      const auto a1 = (const cx<T>*)pre, a2 = (const cx<T>*)Ha, a3 = (const cx<T>*)Hb;        \
      const auto a4 = (const cx<T>*)post, a5 = (const cx<T>*)tw;                               \
      if (si <= kE / 2 && so <= kE / 2)                                                        \
        hipLaunchKernelGGL((k_time_czt_split<T, PP, kE / 2, kE / 2>), grid, block, 0, st, xs,  \
                           o, a1, a2, a3, a4, a5, M, N, L, Ls, rows);                          \
      else                                                                                     \
        hipLaunchKernelGGL((k_time_czt_split<T, PP, kE, kE>), grid, block, 0, st, xs, o, a1,   \
                           a2, a3, a4, a5, M, N, L, Ls, rows);                                 \
      return hipGetLastError();                                                                \
    }                                                                                          \
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
#define CASE(PP)                                                                               \
  case PP:                                                                                     \
    if constexpr ((sizeof(T) * 2 * lds_stride(PP) * ShapeK2<PP>::G <= 160 * 1024)) {                                                         \
      const int n_tiles = (L + ShapeK2<PP>::G - 1) / ShapeK2<PP>::G;                               \
      const long long ng = 1LL * nblocks * pre_n * post_n * n_tiles;                           \
      if (ng <= 0 || ng > 0x7fffffffLL) return hipErrorInvalidValue;                          \
      const dim3 grid((unsigned)ng), block(ShapeK2<PP>::THREADS);                                \
      const bool half = slots_for<PP>(a_in) <= kE / 2 && slots_for<PP>(a_out) <= kE / 2;      \
      if (half)                                                                                \
        hipLaunchKernelGGL((k_axis_czt<T, PP, kE / 2, kE / 2>), grid, block, 0, st,            \
                           (const cx<T>*)in, (cx<T>*)out, (const cx<T>*)pre, (const cx<T>*)H,  \
                           (const cx<T>*)post, (const cx<T>*)tw, a_in, a_out, pre_n, post_n,   \
                           L, nblocks, n_tiles);                                               \
      else                                                                                     \
        hipLaunchKernelGGL((k_axis_czt<T, PP, kE, kE>), grid, block, 0, st,                    \
                           (const cx<T>*)in, (cx<T>*)out, (const cx<T>*)pre, (const cx<T>*)H,  \
                           (const cx<T>*)post, (const cx<T>*)tw, a_in, a_out, pre_n, post_n,   \
                           L, nblocks, n_tiles);                                               \
      return hipGetLastError();                                                                \
    }                                                                                          \
    break;
    FBST_FOR_EACH_P(CASE)
#undef CASE
    default:
      break;
  }
  return hipErrorInvalidValue;
}

// LDS of a spreading workgroup: the smallest of these that holds its grids.
constexpr int kSpreadTiers[3] = {36 * 1024, 72 * 1024, 144 * 1024};

template <typename T>
hipError_t launch_nu_spread(int width, const void* in, void* out, const void* pre, const void* posx,
                            const void* posy, const int* order, int lanes, int M, int nfx, int nfy,
                            double beta, int L, int nblocks, hipStream_t st) {
  constexpr int W = sizeof(T) == 4 ? 8 : 16;
  if (width != W || M < 1 || L < 1 || nblocks < 1 || nfx < 2 * W || nfy < 1 || (nfx & (nfx - 1)) ||
      (nfy & (nfy - 1)) || (nfy > 1 && (!posy || nfy < 2 * W)) || (nfy == 1 && !order) ||
      lanes < 1 || lanes > 16 || (lanes & (lanes - 1)))
    return hipErrorInvalidValue;
  const bool plane = nfy > 1;
  const int per = static_cast<int>(2 * sizeof(T)) * spread_stride(nfx, nfy);
  // frequencies per workgroup: lines up to 16 (a power of two, for the lane
  // mapping); planes 1..4 waves, whichever keeps the most waves resident
  int G = 0, tier = 0, best = 0;
  for (int c = plane ? 4 : 16; c >= 1; c = plane ? c - 1 : c / 2) {
    int t = 0;
    while (t < 3 && c * per > kSpreadTiers[t]) ++t;
    if (t == 3) continue;
    const int waves = (160 * 1024 / kSpreadTiers[t]) * (plane ? c : (c * lanes + 63) / 64);
    if (waves > best) {
      best = waves;
      G = c;
      tier = t;
    }
  }
  if (G < 1) return hipErrorInvalidValue;
  const long long ng = 1LL * nblocks * ((L + G - 1) / G);
  if (ng > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(ng)), block(plane ? 64 * G : G * lanes);
  const T b = static_cast<T>(beta * 1.4426950408889634);   // beta log2(e)
  auto go_line = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, block, 0, st, static_cast<const cx<T>*>(in),
                       static_cast<cx<T>*>(out), static_cast<const cx<T>*>(pre),
                       static_cast<const cx<T>*>(posx), order, M, nfx, G, lanes, b, L, nblocks);
  };
  auto go_plane = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, block, 0, st, static_cast<const cx<T>*>(in),
                       static_cast<cx<T>*>(out), static_cast<const cx<T>*>(pre),
                       static_cast<const cx<T>*>(posx), static_cast<const cx<T>*>(posy), M, nfx,
                       nfy, G, b, L, nblocks);
  };
  if (plane) {
    if (tier == 0) go_plane(k_nu_spread_plane<T, W, kSpreadTiers[0]>);
    else if (tier == 1) go_plane(k_nu_spread_plane<T, W, kSpreadTiers[1]>);
    else go_plane(k_nu_spread_plane<T, W, kSpreadTiers[2]>);
  } else {
    if (tier == 0) go_line(k_nu_spread_line<T, W, kSpreadTiers[0]>);
    else if (tier == 1) go_line(k_nu_spread_line<T, W, kSpreadTiers[1]>);
    else go_line(k_nu_spread_line<T, W, kSpreadTiers[2]>);
  }
  return hipGetLastError();
}

// Fused line stage 1b for oversampled grids of 256..4096 points: G
// frequencies per workgroup (a multiple of the FFT round, within 72 KiB of LDS
// if possible, else 144 KiB); returns hipErrorInvalidValue for other sizes.
template <typename T>
hipError_t launch_nu_line_fused(int width, int P, const void* in, void* w, const void* pre,
                                const void* pos, const int* order, int lanes, const void* corr,
                                const void* tw, int M, int a_out, double beta, int L, int nblocks,
                                hipStream_t st) {
  constexpr int W = sizeof(T) == 4 ? 8 : 16;
  if (width != W || M < 1 || L < 1 || nblocks < 1 || !order || lanes < 1 || lanes > 16 ||
      (lanes & (lanes - 1)) || a_out < 1 || 2 * a_out > P)
    return hipErrorInvalidValue;
  const T b = static_cast<T>(beta * 1.4426950408889634);   // beta log2(e)
  switch (P) {
#define CASE(PP)                                                                                 \
  case PP: {                                                                                     \
    constexpr int NT = 256 / (PP / kE);                                                          \
    const int per = static_cast<int>(2 * sizeof(T)) * fused_stride(PP);                          \
    int G = 16, bytes = 72 * 1024;                                                               \
    while (G > NT && G * per > bytes) G /= 2;                                                    \
    if (G * per > bytes) {                                                                       \
      bytes = 144 * 1024;                                                                        \
      G = 16;                                                                                    \
      while (G > NT && G * per > bytes) G /= 2;                                                  \
    }                                                                                            \
    if (G * per > bytes || G % NT) return hipErrorInvalidValue;                                  \
    const long long ng = 1LL * nblocks * ((L + G - 1) / G);                                      \
    if (ng > 0x7fffffffLL) return hipErrorInvalidValue;                                          \
    auto kern = bytes == 72 * 1024 ? k_nu_line_fused<T, W, PP, 72 * 1024>                        \
                                   : k_nu_line_fused<T, W, PP, 144 * 1024>;                      \
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(ng)), dim3(256), 0, st,                  \
                       static_cast<const cx<T>*>(in), static_cast<cx<T>*>(w),                    \
                       static_cast<const cx<T>*>(pre), static_cast<const cx<T>*>(pos), order,    \
                       static_cast<const cx<T>*>(corr), static_cast<const cx<T>*>(tw), M, G,     \
                       lanes, b, L, nblocks, a_out);                                             \
    return hipGetLastError();                                                                    \
  }
    CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096)
#undef CASE
    default:
      break;
  }
  return hipErrorInvalidValue;
}

// Fused 2-D stage 1b for a 32 x 32 oversampled grid (beam grids up to 16 x 16):
// G = 1..4 frequencies (waves) per workgroup, whichever keeps the most waves
// resident; hipErrorInvalidValue for other grids.
template <typename T>
hipError_t launch_nu_plane_fused(int width, int nfx, int nfy, const void* in, void* w,
                                 const void* pre, const void* posx, const void* posy,
                                 const void* cxs, const void* cys, const void* tw, int M, int bu,
                                 int bv, double beta, int L, int nblocks, hipStream_t st) {
  constexpr int W = sizeof(T) == 4 ? 8 : 16;
  if (width != W || nfx != 32 || nfy != 32 || M < 1 || L < 1 || nblocks < 1 || bu < 1 || bv < 1 ||
      2 * bu > 32 || 2 * bv > 32 || !posy || !cys)
    return hipErrorInvalidValue;
  const int per = static_cast<int>(2 * sizeof(T)) * kPlaneS;
  int G = 0, tier = 0, best = 0;
  for (int c = 4; c >= 1; --c) {
    int tr = 0;
    while (tr < 3 && c * per > kSpreadTiers[tr]) ++tr;
    if (tr == 3) continue;
    const int waves = (160 * 1024 / kSpreadTiers[tr]) * c;
    if (waves > best) {
      best = waves;
      G = c;
      tier = tr;
    }
  }
  if (G < 1) return hipErrorInvalidValue;
  const long long ng = 1LL * nblocks * ((L + G - 1) / G);
  if (ng > 0x7fffffffLL) return hipErrorInvalidValue;
  const T b = static_cast<T>(beta * 1.4426950408889634);   // beta log2(e)
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(ng)), dim3(64 * G), 0, st,
                       static_cast<const cx<T>*>(in), static_cast<cx<T>*>(w),
                       static_cast<const cx<T>*>(pre), static_cast<const cx<T>*>(posx),
                       static_cast<const cx<T>*>(posy), static_cast<const cx<T>*>(cxs),
                       static_cast<const cx<T>*>(cys), static_cast<const cx<T>*>(tw), M, G, bu, bv,
                       b, L, nblocks);
  };
  if (tier == 0) go(k_nu_plane_fused<T, W, kSpreadTiers[0]>);
  else if (tier == 1) go(k_nu_plane_fused<T, W, kSpreadTiers[1]>);
  else go(k_nu_plane_fused<T, W, kSpreadTiers[2]>);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_axis_dft(int P, const void* in, void* out, const void* corr, const void* tw,
                           int a_out, int pre_n, int post_n, int L, int nblocks, hipStream_t st) {
  if (a_out < 1 || 2 * a_out > P || pre_n < 1 || post_n < 1 || L < 1 || nblocks < 1)
    return hipErrorInvalidValue;
  switch (P) {
#define CASE(PP)                                                                               \
  case PP:                                                                                     \
    if constexpr ((sizeof(T) * 2 * lds_stride(PP) * ShapeK2<PP>::G <= 160 * 1024)) {          \
      const int n_tiles = (L + ShapeK2<PP>::G - 1) / ShapeK2<PP>::G;                           \
      const long long ng = 1LL * nblocks * pre_n * post_n * n_tiles;                           \
      if (ng > 0x7fffffffLL) return hipErrorInvalidValue;                                      \
      hipLaunchKernelGGL((k_axis_dft<T, PP>), dim3((unsigned)ng), dim3(ShapeK2<PP>::THREADS), \
                         0, st, (const cx<T>*)in, (cx<T>*)out, (const cx<T>*)corr,             \
                         (const cx<T>*)tw, a_out, pre_n, post_n, L, nblocks);                  \
      return hipGetLastError();                                                                \
    }                                                                                          \
    break;
    FBST_FOR_EACH_P(CASE)
#undef CASE
    default:
      break;
  }
  return hipErrorInvalidValue;
}

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

template <typename T, typename TIN, typename TOUT>
hipError_t launch_toeplitz_fu(int P, const void* w, const OutPtrs& outs, const void* G1,
                              const void* G2, const void* pre3, const void* H3, const void* post3,
                              const void* tw, int B, int L, int N, int nblocks, hipStream_t st) {
  if (nblocks < 1 || nblocks > MAX_LAUNCH_BLOCKS) return hipErrorInvalidValue;
  switch (P) {
#define CASE(PP)                                                                               \
  case PP:                                                                                     \
    if constexpr (fits_lds<T, PP>()) {                                                         \
      if (2 * L > PP) return hipErrorInvalidValue;                                             \
      const dim3 grid(grid_for<PP>(nblocks * B)), block(Shape<PP>::THREADS);                   \
      const int sn = slots_for<PP>(N);                                                         \
      const auto a = (const cx<TIN>*)w;                                                        \
      const auto& o = outs;                                                                    \
      if (sn <= kE / 4)                                                                        \
        hipLaunchKernelGGL((k_toeplitz_fu<T, TIN, TOUT, PP, kE / 4>), grid, block, 0, st, a, o, \
                           (const cx<T>*)G1, (const cx<T>*)G2, (const cx<T>*)pre3,              \
                           (const cx<T>*)H3, (const cx<T>*)post3, (const cx<T>*)tw, B, L, N,    \
                           nblocks);                                                           \
      else if (sn <= kE / 2)                                                                   \
        hipLaunchKernelGGL((k_toeplitz_fu<T, TIN, TOUT, PP, kE / 2>), grid, block, 0, st, a, o, \
                           (const cx<T>*)G1, (const cx<T>*)G2, (const cx<T>*)pre3,              \
                           (const cx<T>*)H3, (const cx<T>*)post3, (const cx<T>*)tw, B, L, N,    \
                           nblocks);                                                           \
      else                                                                                     \
        hipLaunchKernelGGL((k_toeplitz_fu<T, TIN, TOUT, PP, kE>), grid, block, 0, st, a, o,     \
                           (const cx<T>*)G1, (const cx<T>*)G2, (const cx<T>*)pre3,              \
                           (const cx<T>*)H3, (const cx<T>*)post3, (const cx<T>*)tw, B, L, N,    \
                           nblocks);                                                           \
      return hipGetLastError();                                                                \
    }                                                                                          \
    break;
    FBST_FOR_EACH_P(CASE)
#undef CASE
    default:
      break;
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_time_czt<float>(int, const InPtrs&, int, void*, const void*, const void*,
                                           const void*, const void*, int, int, int, hipStream_t);
template hipError_t launch_time_czt<double>(int, const InPtrs&, int, void*, const void*, const void*,
                                           const void*, const void*, int, int, int, hipStream_t);
template hipError_t launch_time_czt_split<float>(int, const InPtrs&, int, void*, const void*,
                                                 const void*, const void*, const void*,
                                                 const void*, int, int, int, int, hipStream_t);
template hipError_t launch_time_czt_split<double>(int, const InPtrs&, int, void*, const void*,
                                                  const void*, const void*, const void*,
                                                  const void*, int, int, int, int, hipStream_t);
template hipError_t launch_axis_czt<float>(int, const void*, void*, const void*, const void*,
                                           const void*, const void*, int, int, int, int, int, int,
                                           hipStream_t);
template hipError_t launch_axis_czt<double>(int, const void*, void*, const void*, const void*,
                                            const void*, const void*, int, int, int, int, int, int,
                                            hipStream_t);
template hipError_t launch_nu_spread<float>(int, const void*, void*, const void*, const void*,
                                            const void*, const int*, int, int, int, int, double,
                                            int, int, hipStream_t);
template hipError_t launch_nu_spread<double>(int, const void*, void*, const void*, const void*,
                                             const void*, const int*, int, int, int, int, double,
                                             int, int, hipStream_t);
template hipError_t launch_nu_line_fused<float>(int, int, const void*, void*, const void*,
                                                const void*, const int*, int, const void*,
                                                const void*, int, int, double, int, int, hipStream_t);
template hipError_t launch_nu_line_fused<double>(int, int, const void*, void*, const void*,
                                                 const void*, const int*, int, const void*,
                                                 const void*, int, int, double, int, int, hipStream_t);
template hipError_t launch_nu_plane_fused<float>(int, int, int, const void*, void*, const void*,
                                                 const void*, const void*, const void*,
                                                 const void*, const void*, int, int, int, double,
                                                 int, int, hipStream_t);
template hipError_t launch_nu_plane_fused<double>(int, int, int, const void*, void*, const void*,
                                                  const void*, const void*, const void*,
                                                  const void*, const void*, int, int, int, double,
                                                  int, int, hipStream_t);
template hipError_t launch_axis_dft<float>(int, const void*, void*, const void*, const void*, int,
                                           int, int, int, int, hipStream_t);
template hipError_t launch_axis_dft<double>(int, const void*, void*, const void*, const void*, int,
                                            int, int, int, int, hipStream_t);
template hipError_t launch_toeplitz_fu<float, float, float>(
    int, const void*, const OutPtrs&, const void*, const void*, const void*, const void*, const void*,
    const void*, int, int, int, int, hipStream_t);
template hipError_t launch_toeplitz_fu<double, float, float>(
    int, const void*, const OutPtrs&, const void*, const void*, const void*, const void*, const void*,
    const void*, int, int, int, int, hipStream_t);
template hipError_t launch_toeplitz_fu<double, double, double>(
    int, const void*, const OutPtrs&, const void*, const void*, const void*, const void*, const void*,
    const void*, int, int, int, int, hipStream_t);

}  // namespace fbst
