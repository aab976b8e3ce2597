// Workgroup-cooperative power-of-two FFTs in LDS for gfx950.
//
// One transform of P points is owned by TT = P / E threads; thread t holds
// E elements in registers, v[s] = x[t + s * TT] (s = 0..E-1), both on entry
// and on exit, so a forward transform, a pointwise product and an inverse
// transform chain without any reordering, and global loads/stores of
// consecutive elements by consecutive threads stay coalesced.
//
// Algorithm: self-sorting Stockham passes of radix R (R = E, then one smaller
// remainder pass).  A pass with span NS performs, for butterfly j
// (j = t + q TT, q = 0..E/R-1), k = j mod NS:
//     a[r] = x[j + r P/R] * w_{NS R}^{r k}     (r = 0..R-1)
//     A = DFT_R(a)
//     y[(j - k) R + k + r NS] = A[r]
// The first pass takes its operands from the registers (j + r P/R is the
// register v[q + r E/R]), the last pass leaves its results in the registers,
// and every pass in between exchanges through LDS, so a transform of
// k passes costs k - 1 LDS round trips.
//
// Pruning: a caller that zero-pads its input declares how many leading
// register slots can be non-zero (NZ_IN); the first pass, whose butterfly
// inputs are exactly the slots, then skips the zero operands.  Outputs the
// caller never reads are removed by dead-code elimination of the last pass.
//
// LDS addresses are padded, i -> i + (i >> 4) (one slot every 16 elements, a
// compile-time choice), which spreads the strided radix-16 writes over the
// banks for complex64.
//
// Twiddles: each pass reads w_{NS R}^{r k} from its own contiguous table,
// laid out [r - 1][k] so that consecutive threads read consecutive entries.
// The tables of size P occupy entries [P, 2P) of one array; the pass with span
// NS starts NS - E entries into it (the pass tables tile the range exactly,
// since (R - 1) NS = NS_next - NS).  Values are computed in float64 on the
// host and rounded once.
//
// Merged twiddles (float32 radix-16 passes after the first, FBST_TW_MERGED):
// the pass's DFT_16 of x_r w^{r k} is taken as 4 x 4 (r = 4 n1 + n2,
// output k' = k1 + 4 k2).  The outer twiddles fold into the two stages:
//   Y[n2][k1]     = sum_n1 x_{4 n1 + n2} psi^{n1} i^{DIR n1 k1},   psi = w^{4 k}
//   X[k1 + 4 k2]  = sum_n2 Y[n2][k1] om^{n2} i^{DIR n2 k2},         om  = w^k w_16^{k1}
// and a 4-point DFT with twiddle om, z_n -> sum_n z_n om^n i^{DIR n k2}, is
// four butterflies x +- c y of the form x +- om^2 y, x +- om y and
// x +- (i^DIR om) y.  With each factor held as (c, t) = (Re f, Im f / Re f),
// x + f y = x + c (y.re - t y.im, y.im + t y.re): two fused multiply-adds for
// the bracket and one per output component, 6 instructions per butterfly in
// place of a complex product (4) and a complex add and subtract (4).  A pass
// therefore takes 192 instead of 220 instructions per radix-16 butterfly (the
// linear-algebra idea is the cosine-scaled twiddle of Linzer and Feig).
// The 15 factors of each k are psi^2, psi, i^-1 psi, then om^2, om, i^-1 om
// for k1 = 0..3 (forward sign), in the [factor][k] layout of the plain
// tables, in entries [TW_MERGED, TW_TABLE) of the same array at the same
// offsets.  |Re f| is held at least 2^-40 so that t stays finite; that moves
// f by less than 1e-12.
#pragma once

#include "cx.h"

namespace fbst {

constexpr int PMAX = 16384;      // largest supported transform size
constexpr int FFT_E = 16;        // elements per thread (radix of the full passes)
constexpr int TW_ENTRIES = 2 * PMAX;
constexpr int TW_MERGED = TW_ENTRIES;        // first entry of the merged tables
constexpr int TW_TABLE = 2 * TW_ENTRIES;     // entries of the whole twiddle array
#ifndef FBST_TW_MERGED
#define FBST_TW_MERGED 1
#endif
// passes that use the merged tables: float32, radix 16, not the first
template <typename T, int R, int NS>
__host__ __device__ constexpr bool merged_pass() {
  return FBST_TW_MERGED && sizeof(T) == 4 && R == 16 && NS > 1;
}

#ifndef FBST_LDS_PAD_SHIFT
#define FBST_LDS_PAD_SHIFT 4
#endif
constexpr int kPadShift = FBST_LDS_PAD_SHIFT;    // one padding slot every 2^kPadShift elements
constexpr int kPadRun = 1 << kPadShift;

__host__ __device__ constexpr int lds_pad(int i) { return i + (i >> kPadShift); }
// per-transform LDS stride in elements: the padded size plus a skew that
// places the transforms of one workgroup (same element index, consecutive
// lanes) in different banks
#ifndef FBST_LDS_SKEW
#define FBST_LDS_SKEW 1
#endif
__host__ __device__ constexpr int lds_stride(int P) { return P + (P >> kPadShift) + FBST_LDS_SKEW; }
// first entry of the twiddle table of the pass with span NS of a P-point transform
__host__ __device__ constexpr int tw_offset(int P, int NS) { return P + NS - FFT_E; }

// Padded LDS slots of the operands of a pass.  The padding is additive over
// multiples of the run length, pad(i + m 2^s) = pad(i) + m (2^s + 1), so every
// operand of a butterfly sits at a compile-time offset from one computed base
// and the accesses use the instruction's immediate offset instead of one
// address register per operand.
template <int P, int R>
__device__ __forceinline__ int read_slot(int j, int r) {
  constexpr int S = P / R;
  if constexpr (S % kPadRun == 0) return lds_pad(j) + r * (S / kPadRun) * (kPadRun + 1);
  else return lds_pad(j + r * S);
}
template <int R, int NS>
__device__ __forceinline__ int write_slot(int base, int r) {
  if constexpr (NS == 1 && kPadRun % R == 0) return lds_pad(base) + r;   // base = j R, r < R
  else if constexpr (NS % kPadRun == 0) return lds_pad(base) + r * (NS / kPadRun) * (kPadRun + 1);
  else return lds_pad(base + r * NS);
}

// ---------------------------------------------------------------------------
// Small DFTs in registers, natural order in and out.  DIR = -1: forward
// (exp(-j ...)); DIR = +1: inverse without scaling.  NZ: inputs [NZ, R) are
// known to be zero.
// ---------------------------------------------------------------------------
namespace detail {
constexpr double kC1 = 0.92387953251128675613;   // cos(pi/8)
constexpr double kS1 = 0.38268343236508977173;   // sin(pi/8)
constexpr double kR2 = 0.70710678118654752440;   // sqrt(2)/2
}  // namespace detail

// a * exp(DIR * j * 2 pi * e / 16)
template <int e, int DIR, typename T>
__device__ __forceinline__ cx<T> tw16(cx<T> a) {
  constexpr int m = ((e % 16) + 16) % 16;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (m == 4) {
    return rot90<DIR>(a);
  } else if constexpr (m == 8) {
    return cx<T>{-a.re, -a.im};
  } else if constexpr (m == 12) {
    return rot90<-DIR>(a);
  } else if constexpr (m % 2 == 0) {
    // odd multiples of pi/4: (+-1 +- j) sqrt(2)/2
    constexpr T r = static_cast<T>(detail::kR2);
    constexpr int c_sign = (m == 2 || m == 14) ? 1 : -1;      // sign of cos
    constexpr int s_sign = (m == 2 || m == 6) ? 1 : -1;       // sign of sin
    constexpr int s = s_sign * DIR;                           // sign of imaginary part of factor
    T re, im;
    if constexpr (c_sign > 0) {
      if constexpr (s > 0) { re = a.re - a.im; im = a.re + a.im; }
      else { re = a.re + a.im; im = a.im - a.re; }
    } else {
      if constexpr (s > 0) { re = -a.re - a.im; im = a.re - a.im; }
      else { re = a.im - a.re; im = -a.re - a.im; }
    }
    return cx<T>{re * r, im * r};
  } else {
    constexpr double cs[16] = {1.0, detail::kC1, detail::kR2, detail::kS1, 0.0, -detail::kS1,
                               -detail::kR2, -detail::kC1, -1.0, -detail::kC1, -detail::kR2,
                               -detail::kS1, 0.0, detail::kS1, detail::kR2, detail::kC1};
    constexpr double sn[16] = {0.0, detail::kS1, detail::kR2, detail::kC1, 1.0, detail::kC1,
                               detail::kR2, detail::kS1, 0.0, -detail::kS1, -detail::kR2,
                               -detail::kC1, -1.0, -detail::kC1, -detail::kR2, -detail::kS1};
    constexpr T c = static_cast<T>(cs[m]);
    constexpr T s = static_cast<T>(DIR * sn[m]);
    return cx<T>{a.re * c - a.im * s, a.re * s + a.im * c};
  }
}

// 4-point DFT in place; inputs [NZ, 4) are zero.
template <int DIR, int NZ, typename T>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  if constexpr (NZ <= 0) {
    a0 = a1 = a2 = a3 = cx<T>{0, 0};
  } else if constexpr (NZ == 1) {
    a1 = a0;
    a2 = a0;
    a3 = a0;
  } else if constexpr (NZ == 2) {
    const cx<T> r1 = rot90<DIR>(a1);
    const cx<T> x0 = a0;
    a0 = x0 + a1;
    a2 = x0 - a1;
    a1 = x0 + r1;
    a3 = x0 - r1;
  } else {
    const cx<T> t0 = (NZ >= 3) ? a0 + a2 : a0, t1 = (NZ >= 3) ? a0 - a2 : a0;
    const cx<T> t2 = (NZ >= 4) ? a1 + a3 : a1;
    const cx<T> t3 = rot90<DIR>((NZ >= 4) ? a1 - a3 : a1);
    a0 = t0 + t2;
    a2 = t0 - t2;
    a1 = t1 + t3;
    a3 = t1 - t3;
  }
}

template <int R, int DIR, int NZ, typename T>
__device__ __forceinline__ void dft(cx<T> (&v)[R]) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    if constexpr (NZ >= 2) {
      const cx<T> a = v[0];
      v[0] = a + v[1];
      v[1] = a - v[1];
    } else {
      v[1] = v[0];
    }
  } else if constexpr (R == 4) {
    dft4<DIR, NZ>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    // n = 2 n1 + n2, k = k1 + 4 k2; input 2 n1 + n2 is non-zero iff < NZ
    dft4<DIR, (NZ + 1) / 2>(v[0], v[2], v[4], v[6]);
    dft4<DIR, NZ / 2>(v[1], v[3], v[5], v[7]);
    v[3] = tw16<2, DIR>(v[3]);
    v[5] = tw16<4, DIR>(v[5]);
    v[7] = tw16<6, DIR>(v[7]);
    cx<T> o[8];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      o[k1] = v[2 * k1] + v[2 * k1 + 1];
      o[k1 + 4] = v[2 * k1] - v[2 * k1 + 1];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = o[i];
  } else if constexpr (R == 16) {
    // n = 4 n1 + n2, k = k1 + 4 k2; input 4 n1 + n2 is non-zero iff < NZ
    dft4<DIR, (NZ + 3) / 4>(v[0], v[4], v[8], v[12]);
    dft4<DIR, (NZ + 2) / 4>(v[1], v[5], v[9], v[13]);
    dft4<DIR, (NZ + 1) / 4>(v[2], v[6], v[10], v[14]);
    dft4<DIR, NZ / 4>(v[3], v[7], v[11], v[15]);
    // Y[n2][k1] sits in v[4 k1 + n2]; multiply by w16^(n2 k1)
    v[5] = tw16<1, DIR>(v[5]);
    v[6] = tw16<2, DIR>(v[6]);
    v[7] = tw16<3, DIR>(v[7]);
    v[9] = tw16<2, DIR>(v[9]);
    v[10] = tw16<4, DIR>(v[10]);
    v[11] = tw16<6, DIR>(v[11]);
    v[13] = tw16<3, DIR>(v[13]);
    v[14] = tw16<6, DIR>(v[14]);
    v[15] = tw16<9, DIR>(v[15]);
    constexpr int nz2 = NZ >= 4 ? 4 : NZ;     // non-zero inputs of the second stage
    dft4<DIR, nz2>(v[0], v[1], v[2], v[3]);
    dft4<DIR, nz2>(v[4], v[5], v[6], v[7]);
    dft4<DIR, nz2>(v[8], v[9], v[10], v[11]);
    dft4<DIR, nz2>(v[12], v[13], v[14], v[15]);
    // X[k1 + 4 k2] sits in v[4 k1 + k2]: transpose 4 x 4
    cx<T> o[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) o[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = o[i];
  } else {
    static_assert(R == 16, "unsupported radix");
  }
}

// x <- x + f y, y <- x - f y with f = c (1 + j t) given as {c, t} (forward
// sign; DIR > 0 applies conj(f))
template <int DIR, typename T>
__host__ __device__ __forceinline__ void bfly_m(cx<T>& x, cx<T>& y, cx<T> f) {
  const T t = DIR < 0 ? f.im : -f.im;
  const T u = fmx(-t, y.im, y.re);
  const T v = fmx(t, y.re, y.im);
  const cx<T> a{fmx(f.re, u, x.re), fmx(f.re, v, x.im)};
  const cx<T> b{fmx(-f.re, u, x.re), fmx(-f.re, v, x.im)};
  x = a;
  y = b;
}

// z_n -> Z[k2] = sum_n z_n om^n i^{DIR n k2}, given om^2, om, i^-1 om (forward
// sign); on return z0..z3 hold Z[0], Z[2], Z[1], Z[3]
template <int DIR, typename T>
__host__ __device__ __forceinline__ void dft4_m(cx<T>& z0, cx<T>& z1, cx<T>& z2, cx<T>& z3,
                                                cx<T> f2, cx<T> f1, cx<T> f3) {
  bfly_m<DIR>(z0, z2, f2);    // z0 + om^2 z2, z0 - om^2 z2
  bfly_m<DIR>(z1, z3, f2);    // z1 + om^2 z3, z1 - om^2 z3
  bfly_m<DIR>(z0, z1, f1);    // Z[0], Z[2]
  bfly_m<DIR>(z2, z3, f3);    // Z[1], Z[3]
}

// DFT_16 of x_r w^{r k} (natural order in and out) from the 15 merged
// factors of k
template <int DIR, typename T, typename F>
__host__ __device__ __forceinline__ void dft16_m(cx<T> (&v)[16], F&& f) {
  // first stage, over n1 for each n2: Y[n2][k1] lands in v[4 br(k1) + n2],
  // br = (0, 2, 1, 3)
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4_m<DIR>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2], f(0), f(1), f(2));
  // second stage, over n2 for each k1: X[k1 + 4 k2] for k2 = 0, 2, 1, 3
  constexpr int br[4] = {0, 2, 1, 3};
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    const int b = 4 * br[k1];
    dft4_m<DIR>(v[b], v[b + 1], v[b + 2], v[b + 3], f(3 + 3 * k1), f(4 + 3 * k1), f(5 + 3 * k1));
  }
  cx<T> o[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int j = 0; j < 4; ++j) o[k1 + 4 * br[j]] = v[4 * br[k1] + j];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = o[i];
}

// ---------------------------------------------------------------------------
// How a pass obtains its twiddles (global loads, L2/L1 latency):
//   TW_LAZY      each one loaded where it is used (fewest live registers; the
//                register-pressure-driven scheduler then tends to serialise
//                the loads, one round trip each);
//   TW_BATCH     the pass's loads issued together after its LDS reads (an
//                empty asm with a memory clobber keeps them above the
//                multiplies), so their latencies overlap;
//   TW_PREFETCH  loaded by the previous pass before its barriers, so their
//                latency overlaps the barrier waits and the LDS exchange (a
//                load issued before a workgroup barrier stays before it: the
//                barrier's release fence orders it); costs one more pass's
//                twiddles in registers across the exchange.
// ---------------------------------------------------------------------------
enum TwiddleMode { TW_LAZY = 0, TW_PREFETCH = 1, TW_BATCH = 2 };


template <typename T, int P, int E, int NS>
struct PassTw {
  static constexpr int REM = P / NS;
  static constexpr int R = (REM >= E) ? E : REM;
  static constexpr int NB = E / R;
  static constexpr int N = (NS > 1) ? NB * (R - 1) : 1;
  cx<T> w[N];
};

// first entry of the table (plain or merged) read by the pass with span NS
template <typename T, int P, int R, int NS>
__device__ __forceinline__ const cx<T>* pass_table(const cx<T>* __restrict__ tw) {
  return tw + (merged_pass<T, R, NS>() ? TW_MERGED : 0) + tw_offset(P, NS);
}

template <typename T, int P, int E, int NS>
__device__ __forceinline__ void load_tw(PassTw<T, P, E, NS>& pt, const cx<T>* __restrict__ tw,
                                        int t) {
  using PT = PassTw<T, P, E, NS>;
  if constexpr (NS > 1) {
    constexpr int TT = P / E;
#pragma unroll
    for (int q = 0; q < PT::NB; ++q) {
      const int k = (t + q * TT) & (NS - 1);
      const cx<T>* twp = pass_table<T, P, PT::R, NS>(tw) + k;
#pragma unroll
      for (int r = 1; r < PT::R; ++r) pt.w[q * (PT::R - 1) + r - 1] = twp[(r - 1) * NS];
    }
  }
}

// ---------------------------------------------------------------------------
// One Stockham pass.  `cur` holds this pass's twiddles; `before_barrier` is
// called once the butterflies are computed and before the first barrier (the
// hook that issues the next pass's twiddle loads).
// ---------------------------------------------------------------------------
// The pass reads its operands from bin (unless FIRST) and writes its results
// to bout (unless LAST); PRE adds the barrier that keeps the writes behind
// every thread's reads of bout's previous contents (needed whenever bout may
// still be read, in particular when bin == bout).
template <typename T, int P, int E, int R, int NS, int DIR, bool FIRST, bool LAST, int NZ_IN,
          int TWM, bool PRE = true, typename Hook>
__device__ __forceinline__ void stockham_pass(cx<T> (&v)[E], const cx<T>* __restrict__ bin,
                                              cx<T>* __restrict__ bout,
                                              const PassTw<T, P, E, NS>& cur,
                                              const cx<T>* __restrict__ tw, int t,
                                              Hook&& before_barrier) {
  constexpr int TT = P / E;
  constexpr int NB = E / R;
  static_assert(E % R == 0, "radix must divide the per-thread element count");
  static_assert(PassTw<T, P, E, NS>::R == R, "twiddle set of another radix");
  cx<T> b[NB][R];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int j = t + q * TT;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if constexpr (FIRST) b[q][r] = v[q + r * NB];
      else b[q][r] = bin[read_slot<P, R>(j, r)];
    }
    if constexpr (NS > 1) {
      const cx<T>* twp = pass_table<T, P, R, NS>(tw) + (j & (NS - 1));
      cx<T> wb[R - 1];
      if constexpr (TWM == TW_BATCH) {
#pragma unroll
        for (int r = 1; r < R; ++r) wb[r - 1] = twp[(r - 1) * NS];
        asm volatile("" ::: "memory");   // issue the loads together (see TW_BATCH)
      }
      auto factor = [&](int i) {
        return TWM == TW_PREFETCH ? cur.w[q * (R - 1) + i] : TWM == TW_BATCH ? wb[i] : twp[i * NS];
      };
      if constexpr (merged_pass<T, R, NS>()) {
        dft16_m<DIR>(b[q], factor);
        continue;
      } else {
#pragma unroll
        for (int r = 1; r < R; ++r) b[q][r] = cmul_dir<DIR>(b[q][r], factor(r - 1));
      }
    }
    if constexpr (FIRST && NB == 1) {
      dft<R, DIR, NZ_IN>(b[q]);
    } else {
      dft<R, DIR, R>(b[q]);
    }
  }
  if constexpr (LAST) {
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r) v[q + r * NB] = b[q][r];
  } else {
    before_barrier();
    if constexpr (PRE) __syncthreads();   // every thread has finished reading the previous contents
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int j = t + q * TT;
      const int k = j & (NS - 1);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) bout[write_slot<R, NS>(base, r)] = b[q][r];
    }
    __syncthreads();   // the new contents are visible to every thread
  }
}

// The same pass over two independent transforms (separate LDS buffers)
// sharing the barriers and the twiddles.
template <typename T, int P, int E, int R, int NS, int DIR, bool FIRST, bool LAST, int NZ_IN,
          int TWM, typename Hook>
__device__ __forceinline__ void stockham_pass2(cx<T> (&v1)[E], cx<T> (&v2)[E],
                                               cx<T>* __restrict__ buf1, cx<T>* __restrict__ buf2,
                                               const PassTw<T, P, E, NS>& cur,
                                               const cx<T>* __restrict__ tw, int t,
                                               Hook&& before_barrier) {
  constexpr int TT = P / E;
  constexpr int NB = E / R;
  static_assert(E % R == 0, "radix must divide the per-thread element count");
  static_assert(PassTw<T, P, E, NS>::R == R, "twiddle set of another radix");
  cx<T> a[NB][R], b[NB][R];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int j = t + q * TT;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if constexpr (FIRST) {
        a[q][r] = v1[q + r * NB];
        b[q][r] = v2[q + r * NB];
      } else {
        a[q][r] = buf1[read_slot<P, R>(j, r)];
        b[q][r] = buf2[read_slot<P, R>(j, r)];
      }
    }
    if constexpr (NS > 1) {
      const cx<T>* twp = pass_table<T, P, R, NS>(tw) + (j & (NS - 1));
      cx<T> wb[R - 1];
      if constexpr (TWM == TW_BATCH) {
#pragma unroll
        for (int r = 1; r < R; ++r) wb[r - 1] = twp[(r - 1) * NS];
        asm volatile("" ::: "memory");
      }
      auto factor = [&](int i) {
        return TWM == TW_PREFETCH ? cur.w[q * (R - 1) + i] : TWM == TW_BATCH ? wb[i] : twp[i * NS];
      };
      if constexpr (merged_pass<T, R, NS>()) {
        dft16_m<DIR>(a[q], factor);
        dft16_m<DIR>(b[q], factor);
        continue;
      } else {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const cx<T> w = factor(r - 1);
          a[q][r] = cmul_dir<DIR>(a[q][r], w);
          b[q][r] = cmul_dir<DIR>(b[q][r], w);
        }
      }
    }
    if constexpr (FIRST && NB == 1) {
      dft<R, DIR, NZ_IN>(a[q]);
      dft<R, DIR, NZ_IN>(b[q]);
    } else {
      dft<R, DIR, R>(a[q]);
      dft<R, DIR, R>(b[q]);
    }
  }
  if constexpr (LAST) {
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        v1[q + r * NB] = a[q][r];
        v2[q + r * NB] = b[q][r];
      }
  } else {
    before_barrier();
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int j = t + q * TT;
      const int k = j & (NS - 1);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        buf1[write_slot<R, NS>(base, r)] = a[q][r];
        buf2[write_slot<R, NS>(base, r)] = b[q][r];
      }
    }
    __syncthreads();
  }
}

// LDS exchanges of a P-point transform (its passes less one)
template <int P, int E>
__host__ __device__ constexpr int fft_exchanges() {
  int n = 0;
  for (int NS = 1; NS < P; NS *= (P / NS >= E ? E : P / NS)) ++n;
  return n - 1;
}

// Pass drivers.  TWM selects how a pass gets its twiddles (TwiddleMode).
// PING: the exchanges alternate between buf and buf + lds_stride(P) (pass XI
// writes buffer XI mod 2), so a pass's writes cannot meet another thread's
// reads of the same pass and need no barrier before them; the first exchange
// keeps it when the transform's last exchange also lands in the first buffer
// (an odd number of exchanges), so that back-to-back transforms stay ordered.
template <typename T, int P, int E, int DIR, int NS, int NZ_IN, int TWM, bool PING = false,
          int XI = 0>
__device__ __forceinline__ void fft_passes(cx<T> (&v)[E], cx<T>* buf, const cx<T>* tw, int t,
                                           PassTw<T, P, E, NS>& cur) {
  constexpr int REM = P / NS;
  constexpr int R = (REM >= E) ? E : REM;
  constexpr bool FIRST = (NS == 1);
  constexpr bool LAST = (REM == R);
  constexpr int S = lds_stride(P);
  const cx<T>* bin = PING ? buf + ((XI + 1) & 1) * S : buf;    // written by pass XI - 1
  cx<T>* bout = PING ? buf + (XI & 1) * S : buf;
  constexpr bool PRE = !PING || (XI == 0 && (fft_exchanges<P, E>() & 1));
  if constexpr (LAST) {
    stockham_pass<T, P, E, R, NS, DIR, FIRST, true, NZ_IN, TWM, PRE>(v, bin, bout, cur, tw, t,
                                                                     [] {});
  } else {
    PassTw<T, P, E, NS * R> nxt;
    stockham_pass<T, P, E, R, NS, DIR, FIRST, false, NZ_IN, TWM, PRE>(v, bin, bout, cur, tw, t,
                                                                      [&] {
      if constexpr (TWM == TW_PREFETCH) load_tw(nxt, tw, t);
    });
    fft_passes<T, P, E, DIR, NS * R, NZ_IN, TWM, PING, XI + 1>(v, buf, tw, t, nxt);
  }
}

template <typename T, int P, int E, int DIR, int NS, int NZ_IN, int TWM>
__device__ __forceinline__ void fft2_passes(cx<T> (&v1)[E], cx<T> (&v2)[E], cx<T>* buf1,
                                            cx<T>* buf2, const cx<T>* tw, int t,
                                            PassTw<T, P, E, NS>& cur) {
  constexpr int REM = P / NS;
  constexpr int R = (REM >= E) ? E : REM;
  constexpr bool FIRST = (NS == 1);
  constexpr bool LAST = (REM == R);
  if constexpr (LAST) {
    stockham_pass2<T, P, E, R, NS, DIR, FIRST, true, NZ_IN, TWM>(v1, v2, buf1, buf2, cur, tw, t,
                                                                [] {});
  } else {
    PassTw<T, P, E, NS * R> nxt;
    stockham_pass2<T, P, E, R, NS, DIR, FIRST, false, NZ_IN, TWM>(v1, v2, buf1, buf2, cur, tw, t,
                                                                 [&] {
      if constexpr (TWM == TW_PREFETCH) load_tw(nxt, tw, t);
    });
    fft2_passes<T, P, E, DIR, NS * R, NZ_IN, TWM>(v1, v2, buf1, buf2, tw, t, nxt);
  }
}

// In-register P-point DFT (DIR = -1) or unscaled inverse (DIR = +1) of the
// transform held by the TT = P / E threads t = 0..TT-1 sharing buf (at least
// lds_stride(P) elements).  v[s] for s >= NZ_IN must be zero on entry.
// Must be reached by every thread of the workgroup (it contains workgroup
// barriers).
// PING: buf holds two transform buffers (2 lds_stride(P) elements) used in
// alternation (fft_passes), one barrier per exchange instead of two; every
// use of them between two such transforms must be a PING transform of the
// same size or be followed by a workgroup barrier.
template <typename T, int P, int E, int DIR, int NZ_IN = E, int TWM = TW_PREFETCH,
          bool PING = false>
__device__ __forceinline__ void fft(cx<T> (&v)[E], cx<T>* buf, const cx<T>* tw, int t) {
  static_assert((P & (P - 1)) == 0 && P >= E && P <= PMAX, "P must be a power of two in [E, PMAX]");
  static_assert(E == FFT_E, "twiddle tables are laid out for FFT_E elements per thread");
  PassTw<T, P, E, 1> none;
  fft_passes<T, P, E, DIR, 1, NZ_IN, TWM, PING>(v, buf, tw, t, none);
}

// Two independent transforms of the same size and direction at once (their
// passes share barriers and twiddle loads); buf1 and buf2 must not overlap.
template <typename T, int P, int E, int DIR, int NZ_IN = E, int TWM = TW_PREFETCH>
__device__ __forceinline__ void fft2(cx<T> (&v1)[E], cx<T> (&v2)[E], cx<T>* buf1, cx<T>* buf2,
                                     const cx<T>* tw, int t) {
  static_assert((P & (P - 1)) == 0 && P >= E && P <= PMAX, "P must be a power of two in [E, PMAX]");
  static_assert(E == FFT_E, "twiddle tables are laid out for FFT_E elements per thread");
  PassTw<T, P, E, 1> none;
  fft2_passes<T, P, E, DIR, 1, NZ_IN, TWM>(v1, v2, buf1, buf2, tw, t, none);
}

}  // namespace fbst
