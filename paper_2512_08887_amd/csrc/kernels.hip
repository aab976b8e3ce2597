// HIP kernels of stage 1 of the FBST hot path for gfx950 (stage 2, K3, is in
// stage2.hip).
//
//   K1 stage 1a  time chirp-z per sensor          (Sec. IV, sum over n of eq. DFT_1)
//   K2 stage 1b  space chirp-z per frequency l     (Sec. IV, sum over m; App. B per axis)
//   non-uniform stage 1b (Sec. IX): spread, fused spread + FFT, per-axis DFT
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
#include "kernel_common.h"

#include <type_traits>

namespace fbst {

namespace {

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
#ifndef FBST_K1S_WAVES
#define FBST_K1S_WAVES 0          // minimum waves per SIMD for the split stage 1a (0: compiler's choice)
#endif
#if FBST_K1S_WAVES > 0
#define FBST_K1S_ATTR __attribute__((amdgpu_waves_per_eu(FBST_K1S_WAVES)))
#else
#define FBST_K1S_ATTR
#endif

// LDS buffers of the split stage 1a: two (the inverses as one dual
// transform) where they fit, else one (float64 at P = 8192)
template <typename T, int P>
constexpr int k1s_bufs() {
  return (FBST_K1S_DUAL && sizeof(T) * 2 * lds_stride(P) * 2 * Shape<P>::G <= 160 * 1024) ? 2 : 1;
}
template <typename T, int P>
constexpr bool k1s_fits() {
  return sizeof(T) * 2 * lds_stride(P) * k1s_bufs<T, P>() * Shape<P>::G <= 160 * 1024;
}

template <typename T, int P, int SI, int SO>
__global__ __launch_bounds__(Shape<P>::THREADS) FBST_K1S_ATTR void k_time_czt_split(
    const InPtrs xs, cx<T>* __restrict__ yhat, const cx<T>* __restrict__ pre,
    const cx<T>* __restrict__ Ha, const cx<T>* __restrict__ Hb, const cx<T>* __restrict__ post,
    const cx<T>* __restrict__ tw, int M, int N, int L, int Ls, int rows) {
  using SH = Shape<P>;
  constexpr int NBUF = k1s_bufs<T, P>();
  __shared__ cx<T> lds[SH::G * NBUF * SH::S];
  const int g = threadIdx.x / SH::TT;
  const int t = threadIdx.x % SH::TT;
  const int row = blockIdx.x * SH::G + g;
  const bool active = row < rows;
  cx<T>* buf = lds + g * NBUF * SH::S;

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
  // the forward transform alternates between the two buffers of the dual
  // inverse where there are two (the dual transform's first exchange keeps
  // its barrier before the writes)
  fft<T, P, kE, -1, SI, FBST_K12_TW, NBUF == 2>(v, buf, tw, t);
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
  if constexpr (NBUF == 2) {
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
template <typename T, int P, int SI, int SO, int WG = FBST_K2_THREADS>
__global__ __launch_bounds__((Shape<P, WG>::THREADS)) FBST_K12_ATTR void k_axis_czt(
    const cx<T>* __restrict__ in, cx<T>* __restrict__ out, const cx<T>* __restrict__ pre,
    const cx<T>* __restrict__ H, const cx<T>* __restrict__ post, const cx<T>* __restrict__ tw,
    int a_in, int a_out, int pre_n, int post_n, int L, int nblocks, int n_tiles) {
  using SH = Shape<P, WG>;
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

}  // namespace

// ---------------------------------------------------------------------------
// Launchers: dispatch the runtime FFT size and slot counts to compiled instances.
// ---------------------------------------------------------------------------

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
                           int post_n, int L, int nblocks, hipStream_t st, int tile) {
  if (tile < 0 || tile > 2) return hipErrorInvalidValue;
  // one instance per workgroup size: tile 0 the default, 1 half as many
  // frequencies per workgroup, 2 twice as many (float32 only)
  auto go = [&](auto wg_tag, auto p_tag) -> hipError_t {
    constexpr int WG = decltype(wg_tag)::value, PP = decltype(p_tag)::value;
    using SH = Shape<PP, WG>;
    if constexpr (sizeof(T) * 2 * lds_stride(PP) * SH::G <= 160 * 1024) {
      const int n_tiles = (L + SH::G - 1) / SH::G;
      const long long ng = 1LL * nblocks * pre_n * post_n * n_tiles;
      if (ng <= 0 || ng > 0x7fffffffLL) return hipErrorInvalidValue;
      const dim3 grid((unsigned)ng), block(SH::THREADS);
      const bool half = slots_for<PP>(a_in) <= kE / 2 && slots_for<PP>(a_out) <= kE / 2;
      if (half)
        hipLaunchKernelGGL((k_axis_czt<T, PP, kE / 2, kE / 2, WG>), grid, block, 0, st,
                           (const cx<T>*)in, (cx<T>*)out, (const cx<T>*)pre, (const cx<T>*)H,
                           (const cx<T>*)post, (const cx<T>*)tw, a_in, a_out, pre_n, post_n, L,
                           nblocks, n_tiles);
      else
        hipLaunchKernelGGL((k_axis_czt<T, PP, kE, kE, WG>), grid, block, 0, st,
                           (const cx<T>*)in, (cx<T>*)out, (const cx<T>*)pre, (const cx<T>*)H,
                           (const cx<T>*)post, (const cx<T>*)tw, a_in, a_out, pre_n, post_n, L,
                           nblocks, n_tiles);
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  };
  using W0 = std::integral_constant<int, FBST_K2_THREADS>;
  using W1 = std::integral_constant<int, FBST_K2_THREADS / 2>;
  using W2 = std::integral_constant<int, FBST_K2_THREADS * 2>;
  if (tile != 0 && sizeof(T) != 4) return hipErrorInvalidValue;
  switch (P) {
#define CASE(PP)                                                                               \
  case PP: {                                                                                   \
    using PT = std::integral_constant<int, PP>;                                                \
    if (tile == 0) return go(W0{}, PT{});                                                      \
    if constexpr (sizeof(T) == 4) {                                                            \
      if (tile == 1) return go(W1{}, PT{});                                                    \
      return go(W2{}, PT{});                                                                   \
    }                                                                                          \
    return hipErrorInvalidValue;                                                               \
  }
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
                                           hipStream_t, int);
template hipError_t launch_axis_czt<double>(int, const void*, void*, const void*, const void*,
                                            const void*, const void*, int, int, int, int, int, int,
                                            hipStream_t, int);
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
}  // namespace fbst
