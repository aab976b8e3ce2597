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

#ifndef FBST_SF_BASE
#define FBST_SF_BASE 64
#endif
constexpr int kBase = FBST_SF_BASE;   // steps done directly (Schur) below this many
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

// FFT size of the window advance at a node of n steps (n1 = n / 2 of them
// first): the windows of n coefficients convolved with Theta_1 (degree n1).
__host__ __device__ inline int advance_size(int n) { return pow2_at_least(n / 2 + n); }

// Scratch (complex128 elements) one solve of L coefficients needs: per depth
// the windows (2 cap), Theta_1 and the result Theta (4 (cap + 1) each) and the
// spectra of Theta_1 at the advance size (4 advance_size(cap)), kept for the
// product Theta_2 Theta_1; plus 12 spectra of the largest FFT size (a window
// advance uses 8 of size <= max_fft, a Theta product 8 of size <= max_fft / 2).
__host__ __device__ inline size_t scratch_elems(int L) {
  int cap[kMaxDepth];
  const int D = depth_caps(L, cap);
  size_t n = 0;
  for (int d = 0; d < D; ++d)
    n += 2 * static_cast<size_t>(cap[d]) + 8 * (static_cast<size_t>(cap[d]) + 1) +
         4 * static_cast<size_t>(advance_size(cap[d]));
  return n + 8 * static_cast<size_t>(max_fft(L));
}

// LDS (or host buffer) elements: the transforms' buffer (max_fft points: one
// transform of the largest size, or several smaller ones at once), plus the
// base case's windows and Theta in two copies.
__host__ __device__ inline int lds_elems(int L) {
  return max_fft(L) + 2 * (2 * kBase + 4 * (kBase + 1));
}

struct Ctx {
  int tid, nth;
  const z* tw;   // tw[k] = exp(-2 pi j k / PM), k < PM / 2
  int PM;
};

// One transform of a batch: dst[i] = s X[off + i] for i < ndst, X the P-point
// DFT (dir -1) or unscaled inverse (dir +1, s = 1 / P; else s = 1) of src
// zero-padded from nsrc points.
struct Xf {
  const z* src;
  int nsrc;
  z* dst;
  int off, ndst;
};

// exp(dir 2 pi j k / Q) from the table, Q a power of two <= PM, k < Q / 2
__host__ __device__ inline z twid(const Ctx& c, int k, int Q, int dir) {
  z w = c.tw[k * (c.PM / Q)];
  if (dir > 0) w.im = -w.im;
  return w;
}

// Radix-2 / radix-4 decimation-in-time passes over g transforms of P points
// at b (bit-reversed order in, natural order out), by lanes lane, lane + W, ...
// of W, with step() between passes.
template <class Step>
__host__ __device__ void dit_passes(z* b, int g, int P, int dir, int lane, int W, const Ctx& c,
                                    Step step) {
  const int bits = ilog2(P);
  int h = 1;
  if (bits & 1) {                         // radix-2: pairs (i, i + 1)
    for (int q = lane; q < g * P / 2; q += W) {
      z* e = b + 2 * q;
      const z a0 = e[0], a1 = e[1];
      e[0] = a0 + a1;
      e[1] = a0 - a1;
    }
    step();
    h = 2;
  }
  for (; h < P; h <<= 2) {                // radix-4: the stages of spans h and 2h at once
    const int quarter = P / 4;
    for (int q = lane; q < g * quarter; q += W) {
      const int t = q / quarter, qq = q - t * quarter;
      const int k = qq % h;
      z* e = b + t * P + (qq / h) * 4 * h + k;
      const z w2 = twid(c, k, 2 * h, dir), w4 = twid(c, k, 4 * h, dir);
      const z a0 = e[0], a1 = cmul(e[h], w2), a2 = e[2 * h], a3 = cmul(e[3 * h], w2);
      const z b0 = a0 + a1, b1 = a0 - a1, b2 = a2 + a3, b3 = a2 - a3;
      const z u2 = cmul(b2, w4);
      z u3 = cmul(b3, w4);
      u3 = dir < 0 ? z{u3.im, -u3.re} : z{-u3.im, u3.re};   // times exp(dir j pi / 2)
      e[0] = b0 + u2;
      e[2 * h] = b0 - u2;
      e[h] = b1 + u3;
      e[3 * h] = b1 - u3;
    }
    step();
  }
}

// Transforms up to this size run one per wave (ordering among the wave's
// lanes only) when the group has several waves.
constexpr int kWaveP = 512;

// cnt transforms of P points (P a power of two): bit-reversed load, radix-4
// decimation-in-time passes (a radix-2 pass first when log2 P is odd), store.
// Small transforms: each wave of the group takes whole transforms in turn
// in its own part of buf, with only sync.wave() between its steps.  Larger
// ones: as many at a time as buf (cap elements) holds, the whole group on
// each, sharing every barrier.
template <class Sync>
__host__ __device__ void xforms(const Xf* jobs, int cnt, int P, int dir, z* buf, int cap,
                                const Ctx& c, Sync sync) {
  const int bits = ilog2(P);
  const int per = cap / P > 0 ? cap / P : 1;
  const double s = dir > 0 ? 1.0 / P : 1.0;
  const int W = c.nth < 64 ? c.nth : 64;
  const int nw = c.nth / W;
  if (nw > 1 && P <= kWaveP && nw * P <= cap) {
    const int lane = c.tid % W, wave = c.tid / W;
    z* b = buf + wave * P;
    for (int j = wave; j < cnt; j += nw) {
      const Xf& jb = jobs[j];
      for (int i = lane; i < P; i += W) b[bitrev(i, bits)] = (i < jb.nsrc) ? jb.src[i] : z{0.0, 0.0};
      sync.wave();
      dit_passes(b, 1, P, dir, lane, W, c, [&] { sync.wave(); });
      for (int i = lane; i < jb.ndst; i += W) jb.dst[i] = b[jb.off + i] * s;
      sync.wave();
    }
    sync();
    return;
  }
  for (int j0 = 0; j0 < cnt; j0 += per) {
    const int g = (cnt - j0 < per) ? cnt - j0 : per;
    for (int i = c.tid; i < g * P; i += c.nth) {
      const int t = i / P, ii = i - t * P;
      const Xf& jb = jobs[j0 + t];
      buf[t * P + bitrev(ii, bits)] = (ii < jb.nsrc) ? jb.src[ii] : z{0.0, 0.0};
    }
    sync();
    dit_passes(buf, g, P, dir, c.tid, c.nth, c, sync);
    for (int i = c.tid; i < g * P; i += c.nth) {
      const int t = i / P, ii = i - t * P;
      const Xf& jb = jobs[j0 + t];
      if (ii < jb.ndst) jb.dst[ii] = buf[t * P + jb.off + ii] * s;
    }
    sync();
  }
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
// The spectra of Theta_1's entries at P = pow2(m + nin) go to ts (4 P), for
// the product Theta_2 Theta_1 when it has the same size.
template <class Sync>
__host__ __device__ void advance(const z* th1, int m, const z* f, const z* g, int nin, int nout,
                                 z* wout, z* ts, z* spec, z* lds, int cap, const Ctx& c,
                                 Sync sync) {
  const int P = pow2_at_least(m + nin);
  z* Ff = spec;
  z* Fg = spec + P;
  z* Af = spec + 2 * P;
  z* Ag = spec + 3 * P;
  const Xf fw[6] = {{f, nin, Ff, 0, P},
                    {g, nin, Fg, 0, P},
                    {th1, m + 1, ts, 0, P},
                    {th1 + (m + 1), m + 1, ts + P, 0, P},
                    {th1 + 2 * (m + 1), m + 1, ts + 2 * P, 0, P},
                    {th1 + 3 * (m + 1), m + 1, ts + 3 * P, 0, P}};
  xforms(fw, 6, P, -1, lds, cap, c, sync);
  // Af = T11 Ff + T12 Fg e^{+2 pi j k / P};  Ag = T21 Ff e^{-2 pi j k / P} + T22 Fg
  const int stride = c.PM / P;
  for (int k = c.tid; k < P; k += c.nth) {
    const int kk = k * stride;   // e^{-2 pi j k / P} from the table (half a turn)
    const z w = (kk < c.PM / 2) ? c.tw[kk] : z{-c.tw[kk - c.PM / 2].re, -c.tw[kk - c.PM / 2].im};
    const z ff = Ff[k], fg = Fg[k];
    Af[k] = cmul(ts[k], ff) + cmul(cmul(ts[P + k], fg), conjg(w));
    Ag[k] = cmul(cmul(ts[2 * P + k], ff), w) + cmul(ts[3 * P + k], fg);
  }
  sync();
  const Xf iv[2] = {{Af, P, wout, m, nout}, {Ag, P, wout + nout, m, nout}};
  xforms(iv, 2, P, +1, lds, cap, c, sync);
}

// Theta = Theta_2 Theta_1 (entries of n2 + 1 and n1 + 1 coefficients) to th,
// n + 1 coefficients per entry (n = n1 + n2).  ts: Theta_1's spectra at size
// pts (from advance), used when pts is this product's size.
template <class Sync>
__host__ __device__ void combine(const z* th2, int n2, const z* th1, int n1, const z* ts, int pts,
                                 z* th, z* spec, z* lds, int cap, const Ctx& c, Sync sync) {
  const int n = n1 + n2;
  const int P = pow2_at_least(n + 1);
  z* T = spec;              // spectra of Theta_2's entries, 4 P
  z* R = spec + 4 * P;      // products, 4 P
  z* A1 = spec + 8 * P;     // Theta_1's spectra when they must be recomputed
  const z* A = ts;
  if (pts != P) {
    const Xf fa[4] = {{th1, n1 + 1, A1, 0, P},
                      {th1 + (n1 + 1), n1 + 1, A1 + P, 0, P},
                      {th1 + 2 * (n1 + 1), n1 + 1, A1 + 2 * P, 0, P},
                      {th1 + 3 * (n1 + 1), n1 + 1, A1 + 3 * P, 0, P}};
    xforms(fa, 4, P, -1, lds, cap, c, sync);
    A = A1;
  }
  const Xf fb[4] = {{th2, n2 + 1, T, 0, P},
                    {th2 + (n2 + 1), n2 + 1, T + P, 0, P},
                    {th2 + 2 * (n2 + 1), n2 + 1, T + 2 * P, 0, P},
                    {th2 + 3 * (n2 + 1), n2 + 1, T + 3 * P, 0, P}};
  xforms(fb, 4, P, -1, lds, cap, c, sync);
  // R_{r,s} = sum_q T_{r,q} A_{q,s}  (entry e = 2 r + s)
  for (int k = c.tid; k < P; k += c.nth) {
    const z t11 = T[k], t12 = T[P + k], t21 = T[2 * P + k], t22 = T[3 * P + k];
    const z a11 = A[k], a12 = A[P + k], a21 = A[2 * P + k], a22 = A[3 * P + k];
    R[k] = cmul(t11, a11) + cmul(t12, a21);
    R[P + k] = cmul(t11, a12) + cmul(t12, a22);
    R[2 * P + k] = cmul(t21, a11) + cmul(t22, a21);
    R[3 * P + k] = cmul(t21, a12) + cmul(t22, a22);
  }
  sync();
  const Xf iv[4] = {{R, P, th, 0, n + 1},
                    {R + P, P, th + (n + 1), 0, n + 1},
                    {R + 2 * P, P, th + 2 * (n + 1), 0, n + 1},
                    {R + 3 * P, P, th + 3 * (n + 1), 0, n + 1}};
  xforms(iv, 4, P, +1, lds, cap, c, sync);
}

// x = A^{-1} e_0 for the first column col (L coefficients, L >= 2).
// scratch: scratch_elems(L); lds: lds_elems(L).  Returns false when a pivot
// eps_k is not positive (then x is unspecified).
// base(f, g, n, th, buf) runs base_case on windows f, g (buf: its LDS area)
// and returns once th is visible to the whole group.
template <class Sync, class Base>
__host__ __device__ bool generator(const z* col, z* x, int L, z* scratch, z* lds, const Ctx& c,
                                   Sync sync, Base base) {
  int cap[kMaxDepth];
  const int D = depth_caps(L, cap);
  z* win[kMaxDepth];
  z* t1[kMaxDepth];
  z* res[kMaxDepth];
  z* ts[kMaxDepth];
  z* p = scratch;
  for (int d = 0; d < D; ++d) {
    win[d] = p;
    p += 2 * static_cast<size_t>(cap[d]);
    t1[d] = p;
    p += 4 * (static_cast<size_t>(cap[d]) + 1);
    res[d] = p;
    p += 4 * (static_cast<size_t>(cap[d]) + 1);
    ts[d] = p;
    p += 4 * static_cast<size_t>(advance_size(cap[d]));
  }
  z* spec = p;
  const int xcap = max_fft(L);    // transform buffer at the start of lds
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
        base(fr.f, fr.g, fr.n, res[d], lds + max_fft(L));
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
      advance(t1[d], n1, fr.f, fr.g, fr.n, n2, win[d + 1], ts[d], spec, lds, xcap, c, sync);
      fr.state = 2;
      st[top + 1] = Frame{n2, 0, 0, win[d + 1], win[d + 1] + n2};
      ++top;
    } else {
      const int n1 = fr.n1, n2 = fr.n - fr.n1;
      combine(res[d + 1], n2, t1[d], n1, ts[d], pow2_at_least(n1 + fr.n), res[d], spec, lds, xcap,
              c, sync);
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

// The same with the base cases run by the whole group.
template <class Sync>
__host__ __device__ bool generator(const z* col, z* x, int L, z* scratch, z* lds, const Ctx& c,
                                   Sync sync) {
  return generator(col, x, L, scratch, lds, c, sync,
                   [&](const z* f, const z* g, int n, z* th, z* buf) {
                     base_case(f, g, n, th, buf, c, sync);
                   });
}

}  // namespace superfast
}  // namespace fbst
