// Superfast solve for the Gohberg-Semencul generator x = A^{-1} e_0 of a
// Hermitian positive definite Toeplitz matrix A (first column c, c_0 real),
// the systems of Sec. V, in O(L log^2 L) operations: the doubling form of the
// Schur algorithm (Ammar and Gragg, "Superfast solution of real positive
// definite Toeplitz systems", SIAM J. Matrix Anal. Appl. 9, 1988; here for
// complex Hermitian matrices), with polynomial products by FFT.
//
// Levinson's predictor polynomials a_k (A_{k+1} a_k = eps_k e_0, a_k[0] = 1)
// and their reverse-conjugates ~a_k(z) = z^k conj(a_k)(1/z) advance by
//     [a_{k+1}; ~a_{k+1}] = [[1, g z], [conj(g), z]] [a_k; ~a_k],
// g = -eta_k / eps_k the reflection coefficient.  The same 2 x 2 polynomial
// matrix maps the residual series F_k = a_k C, G_k = ~a_k C (C the Laurent
// series of c), whose leading coefficients give eta_k ([z^{k+1}] F_k) and
// eps_k ([z^k] G_k).  Schur's form carries only the windows
//     f[i] = [z^{k+1+i}] F_k,  g[i] = [z^{k+i}] G_k,
// one step being  g = -f[0] / g[0],  f <- (f + g g) shifted down by one,
// g <- conj(g) f + g.  m steps need only m coefficients of each window, and
// their product Theta (entries of degree <= m) advances longer windows:
//     f'[i] = sum_j Theta11[j] f[m+i-j] + Theta12[j] g[m+1+i-j],
//     g'[i] = sum_j Theta21[j] f[m-1+i-j] + Theta22[j] g[m+i-j].
// So n steps = n1 steps on the first n1 coefficients (recursively), the
// windows advanced by that Theta_1 (FFT products), n - n1 steps on those
// (recursively), and Theta = Theta_2 Theta_1 (FFT products).  The initial
// windows are f = c[1..L-1], g = c[0..L-2]; after L - 1 steps a_{L-1} =
// Theta11 + Theta12 and x = a_{L-1} / eps with eps = sum_i a_{L-1}[i] conj(c_i).
//
// The code is written for a group of threads that cooperate between
// barriers (tid, nth, sync): the device runs it with one workgroup per system
// (sync = workgroup barrier), the host with one thread (sync does nothing),
// so both execute the same arithmetic.  Every parallel loop writes only its
// own elements and reads only what was written before the last barrier.
#pragma once

#include "cx.h"

namespace fbst {
namespace superfast {

using z = cx<double>;

constexpr int kBase = 32;       // steps done directly (Schur) below this many
constexpr int kMaxDepth = 24;

__host__ __device__ inline int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

__host__ __device__ inline int ilog2(int p) {
  int l = 0;
  while ((1 << l) < p) ++l;
  return l;
}

__host__ __device__ inline int bitrev(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}

__host__ __device__ inline z zdiv(z a, z b) {
  const double d = b.re * b.re + b.im * b.im;
  return z{(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// Largest FFT size the solve uses for L coefficients: the top-level window
// advance convolves L - 1 coefficients with a polynomial of about half that
// length.
__host__ __device__ inline int max_fft(int L) { return pow2_at_least(2 * L); }

// Window capacities per recursion depth: cap[0] = L - 1, cap[d+1] = ceil(cap[d]/2).
__host__ __device__ inline int depth_caps(int L, int* cap) {
  int d = 0;
  cap[0] = L - 1;
  while (cap[d] > kBase && d + 1 < kMaxDepth) {
    cap[d + 1] = (cap[d] + 1) / 2;
    ++d;
  }
  return d + 1;
}

// Scratch (complex128 elements) one solve of L coefficients needs: per depth
// the windows (2 cap), Theta_1 and the result Theta (4 (cap + 1) each), plus 8
// spectra of the largest FFT size (a window advance uses 5 of size <= max_fft,
// a Theta product 9 of size <= max_fft / 2).
__host__ __device__ inline size_t scratch_elems(int L) {
  int cap[kMaxDepth];
  const int D = depth_caps(L, cap);
  size_t n = 0;
  for (int d = 0; d < D; ++d) n += 2 * static_cast<size_t>(cap[d]) + 8 * (static_cast<size_t>(cap[d]) + 1);
  return n + 8 * static_cast<size_t>(max_fft(L));
}

// LDS (or host buffer) elements: one FFT of the largest size, plus the base
// case's windows and Theta in two copies.
__host__ __device__ inline int lds_elems(int L) {
  return max_fft(L) + 2 * (2 * kBase + 4 * (kBase + 1));
}

struct Ctx {
  int tid, nth;
  const z* tw;   // tw[k] = exp(-2 pi j k / PM), k < PM / 2
  int PM;
};

// In-place radix-2 transform of P points held in bit-reversed order in buf,
// result in natural order; dir = -1 forward, +1 inverse (unscaled).
template <class Sync>
__host__ __device__ void fft_inplace(z* buf, int P, int dir, const Ctx& cx_, Sync sync) {
  for (int half = 1; half < P; half <<= 1) {
    const int stride = cx_.PM / (2 * half);
    for (int q = cx_.tid; q < P / 2; q += cx_.nth) {
      const int k = q % half;
      const int i = (q / half) * 2 * half + k;
      z w = cx_.tw[k * stride];
      if (dir > 0) w.im = -w.im;
      const z a = buf[i], b = cmul(buf[i + half], w);
      buf[i] = a + b;
      buf[i + half] = a - b;
    }
    sync();
  }
}

// spec = FFT_P(a zero-padded), a of length na <= P.
template <class Sync>
__host__ __device__ void forward(const z* a, int na, z* spec, z* buf, int P, const Ctx& c,
                                 Sync sync) {
  const int bits = ilog2(P);
  for (int i = c.tid; i < P; i += c.nth) buf[bitrev(i, bits)] = (i < na) ? a[i] : z{0.0, 0.0};
  sync();
  fft_inplace(buf, P, -1, c, sync);
  for (int i = c.tid; i < P; i += c.nth) spec[i] = buf[i];
  sync();
}

// out[i] = IFFT_P(spec)[off + i] for i < n (scaled by 1 / P).
template <class Sync>
__host__ __device__ void inverse(const z* spec, z* out, int off, int n, z* buf, int P, const Ctx& c,
                                 Sync sync) {
  const int bits = ilog2(P);
  for (int i = c.tid; i < P; i += c.nth) buf[bitrev(i, bits)] = spec[i];
  sync();
  fft_inplace(buf, P, +1, c, sync);
  const double s = 1.0 / P;
  for (int i = c.tid; i < n; i += c.nth) out[i] = buf[off + i] * s;
  sync();
}

// n <= kBase Schur steps on windows f, g (length >= n): Theta (4 arrays of
// n + 1 coefficients, [T11 | T12 | T21 | T22]) to th.
template <class Sync>
__host__ __device__ void base_case(const z* f, const z* g, int n, z* th, z* lds, const Ctx& c,
                                   Sync sync) {
  const int W = kBase, T = kBase + 1;
  z* wf[2] = {lds, lds + 2 * W};
  z* wg[2] = {lds + W, lds + 3 * W};
  z* t[2] = {lds + 4 * W, lds + 4 * W + 4 * T};
  for (int i = c.tid; i < n; i += c.nth) {
    wf[0][i] = f[i];
    wg[0][i] = g[i];
  }
  for (int i = c.tid; i < 4 * T; i += c.nth) {
    const int which = i / T, j = i % T;
    t[0][i] = z{((which == 0 || which == 3) && j == 0) ? 1.0 : 0.0, 0.0};
  }
  sync();
  int cur = 0;
  for (int k = 0; k < n; ++k) {
    const z gam = zdiv(z{-wf[cur][0].re, -wf[cur][0].im}, wg[cur][0]);
    const z cg = conjg(gam);
    const int len = n - k;           // window length before the step
    const int nxt = cur ^ 1;
    for (int i = c.tid; i < len - 1; i += c.nth) {
      wf[nxt][i] = wf[cur][i + 1] + cmul(gam, wg[cur][i + 1]);
      wg[nxt][i] = cmul(cg, wf[cur][i]) + wg[cur][i];
    }
    for (int j = c.tid; j <= n; j += c.nth) {
      const z t11 = t[cur][j], t12 = t[cur][T + j];
      const z s21 = (j > 0) ? t[cur][2 * T + j - 1] : z{0.0, 0.0};
      const z s22 = (j > 0) ? t[cur][3 * T + j - 1] : z{0.0, 0.0};
      t[nxt][j] = t11 + cmul(gam, s21);
      t[nxt][T + j] = t12 + cmul(gam, s22);
      t[nxt][2 * T + j] = cmul(cg, t11) + s21;
      t[nxt][3 * T + j] = cmul(cg, t12) + s22;
    }
    sync();
    cur = nxt;
  }
  for (int i = c.tid; i < 4 * (n + 1); i += c.nth) {
    const int which = i / (n + 1), j = i % (n + 1);
    th[i] = t[cur][which * T + j];
  }
  sync();
}

// New windows (nout each, [f | g] to wout) after the m steps of Theta_1 (th1,
// m + 1 coefficients per entry) from windows f, g of length nin = m + nout.
template <class Sync>
__host__ __device__ void advance(const z* th1, int m, const z* f, const z* g, int nin, int nout,
                                 z* wout, z* spec, z* lds, const Ctx& c, Sync sync) {
  const int P = pow2_at_least(m + nin);
  z* Ff = spec;
  z* Fg = spec + P;
  z* S = spec + 2 * P;
  z* Af = spec + 3 * P;
  z* Ag = spec + 4 * P;
  const int stride = c.PM / P;
  forward(f, nin, Ff, lds, P, c, sync);
  forward(g, nin, Fg, lds, P, c, sync);
  for (int e = 0; e < 4; ++e) {
    forward(th1 + e * (m + 1), m + 1, S, lds, P, c, sync);
    // Af = T11 Ff + T12 Fg e^{+2 pi j k / P};  Ag = T21 Ff e^{-2 pi j k / P} + T22 Fg
    for (int k = c.tid; k < P; k += c.nth) {
      // e^{-2 pi j k / P} from the table (k < P; tw holds half a turn)
      const int kk = (k % P) * stride;
      z w = (kk < c.PM / 2) ? c.tw[kk] : z{-c.tw[kk - c.PM / 2].re, -c.tw[kk - c.PM / 2].im};
      z v;
      if (e == 0) v = cmul(S[k], Ff[k]);
      else if (e == 1) v = cmul(cmul(S[k], Fg[k]), conjg(w));
      else if (e == 2) v = cmul(cmul(S[k], Ff[k]), w);
      else v = cmul(S[k], Fg[k]);
      if (e < 2) Af[k] = (e == 0) ? v : Af[k] + v;
      else Ag[k] = (e == 2) ? v : Ag[k] + v;
    }
    sync();
  }
  inverse(Af, wout, m, nout, lds, P, c, sync);
  inverse(Ag, wout + nout, m, nout, lds, P, c, sync);
}

// Theta = Theta_2 Theta_1 (entries of n2 + 1 and n1 + 1 coefficients) to th,
// n + 1 coefficients per entry (n = n1 + n2).
template <class Sync>
__host__ __device__ void combine(const z* th2, int n2, const z* th1, int n1, z* th, z* spec,
                                 z* lds, const Ctx& c, Sync sync) {
  const int n = n1 + n2;
  const int P = pow2_at_least(n + 1);
  z* A = spec;              // spectra of Theta_1's entries, 4 P
  z* R = spec + 4 * P;      // products, 4 P
  for (int e = 0; e < 4; ++e) forward(th1 + e * (n1 + 1), n1 + 1, A + e * P, lds, P, c, sync);
  for (int e = 0; e < 4; ++e) {
    // spectrum of Theta_2 entry e (row r = e / 2, column q = e % 2) into a
    // temporary, then R_{r,s} += T2_{r,q} T1_{q,s}
    z* T = R + 4 * P;      // the fifth scratch spectrum
    forward(th2 + e * (n2 + 1), n2 + 1, T, lds, P, c, sync);
    const int r = e / 2, q = e % 2;
    for (int k = c.tid; k < P; k += c.nth)
      for (int s = 0; s < 2; ++s) {
        const z v = cmul(T[k], A[(2 * q + s) * P + k]);
        z* dst = R + (2 * r + s) * P;
        dst[k] = (q == 0) ? v : dst[k] + v;
      }
    sync();
  }
  for (int e = 0; e < 4; ++e) inverse(R + e * P, th + e * (n + 1), 0, n + 1, lds, P, c, sync);
}

// x = A^{-1} e_0 for the first column col (L coefficients, L >= 2).
// scratch: scratch_elems(L); lds: lds_elems(L).  Returns false when a pivot
// eps_k is not positive (then x is unspecified).
template <class Sync>
__host__ __device__ bool generator(const z* col, z* x, int L, z* scratch, z* lds, const Ctx& c,
                                   Sync sync) {
  int cap[kMaxDepth];
  const int D = depth_caps(L, cap);
  z* win[kMaxDepth];
  z* t1[kMaxDepth];
  z* res[kMaxDepth];
  z* p = scratch;
  for (int d = 0; d < D; ++d) {
    win[d] = p;
    p += 2 * static_cast<size_t>(cap[d]);
    t1[d] = p;
    p += 4 * (static_cast<size_t>(cap[d]) + 1);
    res[d] = p;
    p += 4 * (static_cast<size_t>(cap[d]) + 1);
  }
  z* spec = p;
  struct Frame {
    int n, n1, state;
    const z* f;
    const z* g;
  };
  Frame st[kMaxDepth];
  int top = 0;
  st[0] = Frame{L - 1, 0, 0, col + 1, col};
  while (top >= 0) {
    Frame& fr = st[top];
    const int d = top;
    if (fr.state == 0) {
      if (fr.n <= kBase) {
        base_case(fr.f, fr.g, fr.n, res[d], lds + max_fft(L), c, sync);
        --top;
        continue;
      }
      fr.n1 = fr.n / 2;
      fr.state = 1;
      st[top + 1] = Frame{fr.n1, 0, 0, fr.f, fr.g};
      ++top;
    } else if (fr.state == 1) {
      const int n1 = fr.n1, n2 = fr.n - fr.n1;
      for (int i = c.tid; i < 4 * (n1 + 1); i += c.nth) t1[d][i] = res[d + 1][i];
      sync();
      advance(t1[d], n1, fr.f, fr.g, fr.n, n2, win[d + 1], spec, lds, c, sync);
      fr.state = 2;
      st[top + 1] = Frame{n2, 0, 0, win[d + 1], win[d + 1] + n2};
      ++top;
    } else {
      const int n1 = fr.n1, n2 = fr.n - fr.n1;
      combine(res[d + 1], n2, t1[d], n1, res[d], spec, lds, c, sync);
      --top;
    }
  }
  // a = Theta11 + Theta12 (L coefficients); eps = sum_i a[i] conj(c_i)
  const z* th = res[0];
  const int n = L - 1;
  for (int i = c.tid; i < L; i += c.nth) x[i] = th[i] + th[(n + 1) + i];
  sync();
  z eps{0.0, 0.0};
  for (int i = 0; i < L; ++i) eps = eps + cmulc(x[i], col[i]);
  sync();
  if (!(eps.re > 0.0)) return false;
  for (int i = c.tid; i < L; i += c.nth) x[i] = zdiv(x[i], eps);
  sync();
  return true;
}

}  // namespace superfast
}  // namespace fbst
