// FP64 host plan builder: validation, chirp tables, chirp-kernel spectra,
// Toeplitz generators and Gohberg-Semencul spectra.
#include "plan.h"
#include "superfast.h"

#include <sched.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <mutex>
#include <thread>

#include "fft_lds.h"

namespace fbst {

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

zd cis(double ph) { return zd(std::cos(ph), std::sin(ph)); }

// exp(j pi x), with x reduced modulo 2 exactly before the trigonometric call
zd cispi(double x) {
  const double r = std::fmod(x, 2.0);
  return zd(std::cos(kPi * r), std::sin(kPi * r));
}

int next_pow2(long long n) {
  long long p = 1;
  while (p < n) p <<= 1;
  return static_cast<int>(std::min<long long>(p, 1LL << 30));
}

// sum_{n=0}^{K-1} exp(j (phi0 + n phi))
zd geometric_sum(int K, double phi0, double phi) {
  const double s = std::sin(0.5 * phi);
  if (s == 0.0) {
    // phi is a multiple of 2 pi (to the last bit): every term equals exp(j phi0)
    return cis(phi0) * static_cast<double>(K);
  }
  const double ratio = std::sin(0.5 * K * phi) / s;
  return cis(phi0 + 0.5 * (K - 1) * phi) * ratio;
}

// Default grid of eq. (thetab): odd count (2b - B - 1)/(B - 1), even count
// (2b - B - 1)/B, b = 1..B; one beam at broadside.
void default_grid(int B, double* u0, double* du) {
  if (B <= 1) {
    *u0 = 0.0;
    *du = 0.0;
  } else if (B % 2 == 1) {
    *u0 = -1.0;
    *du = 2.0 / (B - 1);
  } else {
    *u0 = (1.0 - B) / B;
    *du = 2.0 / B;
  }
}

// Circularly placed chirp kernel exp(j * coef * (k + shift)^2) for
// k in [kmin, kmax], put at index k mod P; returns its scaled spectrum FFT/P.
// phase/pi = coef_pi * (k + shift)^2 evaluated with an exact integer square.
std::vector<zd> kernel_spectrum_int(int P, long long kmin, long long kmax, long long shift,
                                    double coef_pi) {
  std::vector<zd> h(P, zd(0.0, 0.0));
  for (long long k = kmin; k <= kmax; ++k) {
    const long long q = k + shift;
    const double q2 = static_cast<double>(q * q);
    const long long idx = ((k % P) + P) % P;
    h[idx] = cispi(coef_pi * q2);
  }
  fft64(h.data(), P, -1);
  const double s = 1.0 / P;
  for (auto& z : h) z *= s;
  return h;
}

// Run fn(i0, i1) over [0, n) on the hardware threads when the work is large.
int cpu_threads() {
  cpu_set_t set;
  if (sched_getaffinity(0, sizeof(set), &set) == 0) return std::max(1, CPU_COUNT(&set));
  return std::max(1, static_cast<int>(std::thread::hardware_concurrency()));
}

template <typename F>
void parallel_for(int n, long long cost, F&& fn) {
  const int hw = cpu_threads();
  const int nthreads = std::min({hw, n, 64});
  if (nthreads <= 1 || cost < 4'000'000LL) {
    fn(0, n);
    return;
  }
  std::vector<std::thread> th;
  const int per = (n + nthreads - 1) / nthreads;
  for (int i = 0; i < nthreads; ++i) {
    const int a = i * per, b = std::min(n, a + per);
    if (a < b) th.emplace_back([&fn, a, b] { fn(a, b); });
  }
  for (auto& x : th) x.join();
}

void build_axis(const Params& p, int a_in, int a_out, double pos0, double d_samples, double u0,
                double du, int P, AxisTables* ax) {
  const int L = p.L;
  ax->a_in = a_in;
  ax->a_out = a_out;
  ax->P = P;
  ax->pre.assign(static_cast<size_t>(a_in) * L, zd());
  ax->H.assign(static_cast<size_t>(P) * L, zd());
  ax->post.assign(static_cast<size_t>(a_out) * L, zd());
  const double lp0 = 1.0 - 0.5 * L;
  // frequencies are independent: split them over the host threads
  parallel_for(L, 1LL * L * P * 16, [&](int l0, int l1) {
  std::vector<zd> h(P);
  for (int l = l0; l < l1; ++l) {
    const double lp = l + lp0;
    const double rho = 2.0 * kPi * (p.fc * p.ts + p.eps * lp / L);   // rad per (sample of delay)
    const double theta = rho * d_samples * du;
    for (int i = 0; i < a_in; ++i) {
      const double di = i;
      ax->pre[static_cast<size_t>(i) * L + l] = cis(rho * d_samples * u0 * di + 0.5 * theta * di * di);
    }
    std::fill(h.begin(), h.end(), zd());
    for (int k = -(a_in - 1); k <= a_out - 1; ++k) {
      const double dk = k;
      h[((k % P) + P) % P] = cis(-0.5 * theta * dk * dk);
    }
    fft64(h.data(), P, -1);
    for (int i = 0; i < P; ++i) ax->H[static_cast<size_t>(i) * L + l] = h[i] / static_cast<double>(P);
    for (int a = 0; a < a_out; ++a) {
      const double da = a;
      ax->post[static_cast<size_t>(a) * L + l] =
          cis(rho * d_samples * pos0 * (u0 + da * du) + 0.5 * theta * da * da);
    }
  }
  });
}

// beta = A^{-1} r through the Gohberg-Semencul form with generator x
// (x0 = x[0] real), circulant-embedded in P >= 2L - 1 points; float64.
void gs_apply(const std::vector<zd>& x, const std::vector<zd>& r, int L, int P, std::vector<zd>* out) {
  std::vector<zd> g1(P), g2(P), v(P), a(P), b(P);
  std::copy(x.begin(), x.end(), g1.begin());
  for (int i = 1; i < L; ++i) g2[i] = std::conj(x[L - i]);
  std::copy(r.begin(), r.end(), v.begin());
  fft64(g1.data(), P, -1);
  fft64(g2.data(), P, -1);
  fft64(v.data(), P, -1);
  for (int i = 0; i < P; ++i) {
    a[i] = std::conj(g1[i]) * v[i];
    b[i] = std::conj(g2[i]) * v[i];
  }
  fft64(a.data(), P, +1);
  fft64(b.data(), P, +1);
  for (int i = 0; i < P; ++i) {
    const bool keep = i < L;
    a[i] = keep ? a[i] / static_cast<double>(P) : zd();
    b[i] = keep ? b[i] / static_cast<double>(P) : zd();
  }
  fft64(a.data(), P, -1);
  fft64(b.data(), P, -1);
  for (int i = 0; i < P; ++i) v[i] = g1[i] * a[i] - g2[i] * b[i];
  fft64(v.data(), P, +1);
  out->resize(L);
  const double s = 1.0 / (static_cast<double>(P) * x[0].real());
  for (int i = 0; i < L; ++i) (*out)[i] = v[i] * s;
}

// One step of iterative refinement of x ~ A^{-1} e_0: the residual
// e_0 - A x is formed exactly enough in long double (O(L^2)), and the
// correction solves A dx = r with the Gohberg-Semencul form of x itself.
// Levinson's forward error grows like cond(A) u; the refined generator is
// accurate to a few u even when cond(A) ~ 1e9 (delta of 1e-5).
void refine_generator(const zd* col, int L, int P, std::vector<zd>* x) {
  using ld = long double;
  std::vector<zd> r(L);
  for (int i = 0; i < L; ++i) {
    ld re = (i == 0) ? 1.0L : 0.0L, im = 0.0L;
    for (int k = 0; k < L; ++k) {
      // A[i][k] = col[i-k] for i >= k, conj(col[k-i]) otherwise
      const zd a = (i >= k) ? col[i - k] : std::conj(col[k - i]);
      const ld ar = a.real(), ai = a.imag(), xr = (*x)[k].real(), xi = (*x)[k].imag();
      re -= ar * xr - ai * xi;
      im -= ar * xi + ai * xr;
    }
    r[i] = zd(static_cast<double>(re), static_cast<double>(im));
  }
  std::vector<zd> dx;
  gs_apply(*x, r, L, P, &dx);
  for (int i = 0; i < L; ++i) (*x)[i] += dx[i];
  (*x)[0] = zd((*x)[0].real(), 0.0);
}

// sum_m exp(j (ax xs_m + ay ys_m)) over the elements, positions in samples of
// delay per unit direction cosine and ax, ay in rad per sample: closed-form
// geometric sums per axis for a line or grid, the direct sum otherwise.
zd sensor_sum(const Params& p, double ax, double ay) {
  if (p.kind == FBST_ARBITRARY) {
    double re = 0.0, im = 0.0;
    for (int m = 0; m < p.M; ++m) {
      const double ph = ax * (p.px[m] / p.ts) + ay * (p.py[m] / p.ts);
      re += std::cos(ph);
      im += std::sin(ph);
    }
    return zd(re, im);
  }
  const double thx = ax * (p.dx / p.ts);
  zd s = geometric_sum(p.mx, thx * p.x0, thx);
  if (p.kind == FBST_GRID) {
    const double thy = ay * (p.dy / p.ts);
    s *= geometric_sum(p.my, thy * p.y0, thy);
  }
  return s;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int n, std::vector<double>* x, std::vector<double>* w) {
  x->assign(n, 0.0);
  w->assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;                 // P_0, P_1
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);  // P_n'(z)
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    (*x)[i] = -z;
    (*x)[n - 1 - i] = z;
    (*w)[i] = (*w)[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Exponential-of-semicircle spreading kernel phi(z) = exp(beta (sqrt(1 - z^2) - 1))
// on |z| <= 1 (Barnett, Magland, af Klinteberg, SIAM J. Sci. Comput. 2019).
double es_kernel(double beta, double z) {
  const double q = 1.0 - z * z;
  return q > 0.0 ? std::exp(beta * (std::sqrt(q) - 1.0)) : (q == 0.0 ? std::exp(-beta) : 0.0);
}

// Deconvolution factors of one axis: mode k = a - a_out/2 of an nf-point grid
// spread with a w-point kernel is divided by (nf / 2 pi) psi^(k), psi^ the
// Fourier transform of the kernel in radians: psi^(k) = (pi w / nf)
// int_{-1}^{1} phi(z) cos(k pi w z / nf) dz (Gauss-Legendre, 4w + 32 nodes).
std::vector<zd> nu_deconvolution(int a_out, int nf, int w, double beta) {
  std::vector<double> zq, wq;
  gauss_legendre(4 * w + 32, &zq, &wq);
  std::vector<zd> c(a_out);
  for (int a = 0; a < a_out; ++a) {
    const double k = a - a_out / 2;
    double s = 0.0;
    for (size_t i = 0; i < zq.size(); ++i)
      s += wq[i] * es_kernel(beta, zq[i]) * std::cos(k * kPi * w * zq[i] / nf);
    c[a] = zd(1.0 / (0.5 * w * s), 0.0);
  }
  return c;
}

// Type-1 non-uniform FFT tables of stage 1b (Sec. IX, eq. DFT_non_unif).  With
// centre mode a_c = bu / 2 (c_c = bv / 2) and f_l = f_c T_s + eps l' / L
// (cycles per sample of delay), the phase f_l 2 pi (u_a xs_m + v_c ys_m) of
// beam (a, c) splits into the centre-direction phase (nu_pre) and
// (a - a_c) s_x + (c - c_c) s_y with s_x = 2 pi f_l du xs_m,
// s_y = 2 pi f_l dv ys_m: one type-1 NUFFT per l over the modes of the
// beam grid, with the points at s_x / 2 pi mod 1 of the oversampled grid.
// Phases and positions are reduced in long double.
void build_nonuniform(const Params& p, HostTables* t) {
  const int M = p.M, L = p.L, w = p.nuw;
  const int nfx = p.p2x, nfy = p.p2y;
  const bool two_d = nfy > 0;
  const long double lp0 = 1.0L - 0.5L * L;
  const long double uc = static_cast<long double>(p.u0) + static_cast<long double>(p.bu / 2) * p.du;
  const long double vc = two_d ? static_cast<long double>(p.v0) + static_cast<long double>(p.bv / 2) * p.dv
                               : static_cast<long double>(p.v0);
  t->nu_pre.assign(static_cast<size_t>(M) * L, zd());
  t->nu_posx.assign(static_cast<size_t>(M) * L, zd());
  if (two_d) t->nu_posy.assign(static_cast<size_t>(M) * L, zd());
  auto frac = [](long double v) { return v - std::floor(v); };
  auto position = [&](long double cyc, int nf) {
    const long double g = frac(cyc) * nf;
    long double jf = std::floor(g);
    long double f = g - jf;
    if (f >= 1.0L) { f = 0.0L; jf += 1.0L; }
    long long j0 = (static_cast<long long>(jf) - w / 2 + 1) % nf;
    if (j0 < 0) j0 += nf;
    return zd(static_cast<double>(f), static_cast<double>(j0));
  };
  std::vector<int> j0x(two_d ? 0 : static_cast<size_t>(M) * L);
  parallel_for(M, 1LL * M * L * 64, [&](int m0, int m1) {
    for (int m = m0; m < m1; ++m) {
      const long double xs = static_cast<long double>(p.px[m]) / p.ts;
      const long double ys = static_cast<long double>(p.py[m]) / p.ts;
      for (int l = 0; l < L; ++l) {
        const long double fl = static_cast<long double>(p.fc) * p.ts +
                               static_cast<long double>(p.eps) * (l + lp0) / L;
        const size_t i = static_cast<size_t>(m) * L + l;
        t->nu_pre[i] = cis(2.0 * kPi * static_cast<double>(frac(fl * (uc * xs + vc * ys))));
        t->nu_posx[i] = position(fl * static_cast<long double>(p.du) * xs, nfx);
        if (two_d) t->nu_posy[i] = position(fl * static_cast<long double>(p.dv) * ys, nfy);
        else j0x[i] = static_cast<int>(t->nu_posx[i].imag());
      }
    }
  });
  // Line of beams: lanes per frequency of the spread.  Lane r takes the
  // elements order[r C + s] (C = ceil(M / R)) for s = 0, 1, ...; R is the
  // largest of 16, 8, 4, 2 for which, at every frequency and step s, the
  // w-cell supports of those elements are pairwise disjoint on the periodic
  // grid (else 1: one lane per frequency).
  t->nu_order.assign(M, 0);
  t->nu_lanes = 1;
  if (!two_d) {
    for (int m = 0; m < M; ++m) t->nu_order[m] = m;
    std::stable_sort(t->nu_order.begin(), t->nu_order.end(),
                     [&](int a, int b) { return p.px[a] < p.px[b]; });
    for (int R = 16; R > 1 && t->nu_lanes == 1; R /= 2) {
      const int C = (M + R - 1) / R;
      if (C * (R - 1) >= M) continue;             // a lane would have no elements at all
      std::atomic<bool> good{true};
      parallel_for(L, 1LL * L * C * R * 4, [&](int l0, int l1) {
        std::vector<int> v(R);
        for (int l = l0; l < l1 && good.load(); ++l)
          for (int st = 0; st < C; ++st) {
            int n = 0;
            for (int r = 0; r < R; ++r) {
              const int k = r * C + st;
              if (k < M) v[n++] = j0x[static_cast<size_t>(t->nu_order[k]) * L + l];
            }
            std::sort(v.begin(), v.begin() + n);
            bool ok = n < 2 || v[0] + nfx - v[n - 1] >= w;
            for (int a = 1; a < n && ok; ++a) ok = v[a] - v[a - 1] >= w;
            if (!ok) {
              good = false;
              break;
            }
          }
      });
      if (good) t->nu_lanes = R;
    }
  }
  t->nu_cx = nu_deconvolution(p.bu, nfx, w, p.nu_beta);
  if (two_d) t->nu_cy = nu_deconvolution(p.bv, nfy, w, p.nu_beta);
}

}  // namespace

double pos_x(const Params& p, int m) {
  if (p.kind == FBST_ARBITRARY) return p.px[m] / p.ts;
  const int k = (p.kind == FBST_GRID) ? m / p.my : m;
  return (p.x0 + k) * (p.dx / p.ts);
}

double pos_y(const Params& p, int m) {
  if (p.kind == FBST_ARBITRARY) return p.py[m] / p.ts;
  if (p.kind != FBST_GRID) return 0.0;
  return (p.y0 + m % p.my) * (p.dy / p.ts);
}

void fft64(zd* a, int n, int sign) {
  // iterative radix-2, bit-reversed input order, twiddles from direct cos/sin
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  std::vector<zd> w(n / 2 > 0 ? n / 2 : 1);
  for (int k = 0; k < n / 2; ++k) w[k] = cis(sign * 2.0 * kPi * k / n);
  for (int len = 2; len <= n; len <<= 1) {
    const int half = len >> 1;
    const int step = n / len;
    for (int i = 0; i < n; i += len) {
      for (int k = 0; k < half; ++k) {
        const zd u = a[i + k];
        const zd v = a[i + k + half] * w[k * step];
        a[i + k] = u + v;
        a[i + k + half] = u - v;
      }
    }
  }
}

bool levinson_first_column(const zd* col, int L, zd* x) {
  // T a_k = e_0 * err_k for the leading (k+1) x (k+1) block, a_k[0] = 1;
  // a_{k+1} = [a_k; 0] - g [0; J conj(a_k)], g = eta / err,
  // eta = sum_i col[k+1-i] a_k[i], err_{k+1} = err_k - g conj(eta).
  std::vector<zd> a(L, zd());
  a[0] = 1.0;
  double err = col[0].real();
  if (!(err > 0.0)) return false;
  for (int k = 0; k + 1 < L; ++k) {
    zd eta = 0.0;
    for (int i = 0; i <= k; ++i) eta += col[k + 1 - i] * a[i];
    const zd g = eta / err;
    // pairwise in-place update of a[i] and a[k+1-i]
    for (int i = 0, j = k + 1; i <= j; ++i, --j) {
      const zd ai = a[i], aj = a[j];
      if (i == j) {
        a[i] = ai - g * std::conj(aj);
      } else {
        a[i] = ai - g * std::conj(aj);
        a[j] = aj - g * std::conj(ai);
      }
    }
    err -= (g * std::conj(eta)).real();
    if (!(err > 0.0)) return false;
  }
  for (int i = 0; i < L; ++i) x[i] = a[i] / err;
  return true;
}

bool levinson_real(const double* col, int L, double* x) {
  // The real symmetric case of levinson_first_column.
  std::vector<double> a(L, 0.0);
  a[0] = 1.0;
  double err = col[0];
  if (!(err > 0.0)) return false;
  for (int k = 0; k + 1 < L; ++k) {
    double eta = 0.0;
    for (int i = 0; i <= k; ++i) eta += col[k + 1 - i] * a[i];
    const double g = eta / err;
    for (int i = 0, j = k + 1; i <= j; ++i, --j) {
      const double ai = a[i], aj = a[j];
      a[i] = ai - g * aj;
      if (i != j) a[j] = aj - g * ai;
    }
    err -= g * eta;
    if (!(err > 0.0)) return false;
  }
  for (int i = 0; i < L; ++i) x[i] = a[i] / err;
  return true;
}

// Largest eigenvalue of the L x L time Gram T[l][k] = sum_{n<N} exp(-j kappa
// (l - k) n), kappa = 2 pi eps / L (the Gram of Sec. V with a single element
// at the origin), by power iteration with circulant-embedded products of
// P >= 2L - 1 points; the Rayleigh quotient of the last iterate.
double time_gram_lmax(int N, int L, double eps) {
  const int P = next_pow2(2LL * L - 1);
  const double kappa = 2.0 * kPi * eps / L;
  std::vector<zd> spec(P, zd()), v(L), buf(P);
  for (int d = 0; d < L; ++d) {
    const zd c = geometric_sum(N, 0.0, -kappa * d);
    spec[d] = c;
    if (d > 0) spec[P - d] = std::conj(c);
  }
  fft64(spec.data(), P, -1);
  // deterministic start with components along every eigenvector
  unsigned long long s = 0x9e3779b97f4a7c15ULL;
  for (int l = 0; l < L; ++l) {
    s = s * 6364136223846793005ULL + 1442695040888963407ULL;
    v[l] = zd(0.5 + static_cast<double>(s >> 11) * 0x1.0p-53, 0.0);
  }
  double lam = 0.0;
  for (int it = 0; it < 40; ++it) {
    double nv = 0.0;
    for (int l = 0; l < L; ++l) nv += std::norm(v[l]);
    nv = std::sqrt(nv);
    std::fill(buf.begin(), buf.end(), zd());
    for (int l = 0; l < L; ++l) buf[l] = v[l] / nv;
    fft64(buf.data(), P, -1);
    for (int i = 0; i < P; ++i) buf[i] *= spec[i];
    fft64(buf.data(), P, +1);
    double rq = 0.0;
    for (int l = 0; l < L; ++l) {
      const zd tv = buf[l] / static_cast<double>(P);
      rq += (std::conj(v[l] / nv) * tv).real();
      v[l] = tv;
    }
    lam = rq;
  }
  return lam;
}

// The beam grid of p (kind and B already set) from fbst_grid; NULL selects
// the eq. (thetab) grid of a line.
fbst_status resolve_grid(Params* pp, const fbst_grid* grid, std::string* msg) {
  Params& p = *pp;
  const int B = p.B;
  if (!grid) {
    if (p.kind == FBST_GRID) {
      *msg = "a grid geometry needs an explicit beam grid (bu x bv)";
      return FBST_E_INVALID;
    }
    p.bu = B;
    p.bv = 1;
    default_grid(B, &p.u0, &p.du);
  } else {
    p.bu = grid->bu;
    p.bv = grid->bv;
    if (p.bu < 1 || p.bv < 1 || 1LL * p.bu * p.bv != B) {
      *msg = "grid needs bu * bv == B";
      return FBST_E_INVALID;
    }
    if (p.kind == FBST_LINE && p.bv != 1) {
      *msg = "a line needs bv == 1";
      return FBST_E_INVALID;
    }
    if (grid->du == 0.0) default_grid(p.bu, &p.u0, &p.du);
    else { p.u0 = grid->u0; p.du = grid->du; }
    if (p.kind != FBST_LINE) {
      if (grid->dv == 0.0) default_grid(p.bv, &p.v0, &p.dv);
      else { p.v0 = grid->v0; p.dv = grid->dv; }
    }
    if (!std::isfinite(p.u0) || !std::isfinite(p.du) || !std::isfinite(p.v0) || !std::isfinite(p.dv)) {
      *msg = "grid values must be finite";
      return FBST_E_INVALID;
    }
  }
  return FBST_OK;
}

fbst_status resolve_params(int M, int N, int B, const fbst_geometry* geom, const fbst_band* band,
                           const fbst_grid* grid, const fbst_options* opt, Params* out,
                           std::string* msg) {
  Params p;
  if (M < 1 || N < 1 || B < 1) {
    *msg = "M, N and B must be >= 1";
    return FBST_E_INVALID;
  }
  if (!band) {
    *msg = "band must not be NULL";
    return FBST_E_INVALID;
  }
  if (!(band->fc >= 0.0) || !(band->omega > 0.0) || !(band->ts > 0.0) ||
      band->ts > 1.0 / (2.0 * band->omega) * (1.0 + 1e-12) || !std::isfinite(band->fc)) {
    *msg = "band needs fc >= 0, omega > 0 and 0 < ts <= 1/(2 omega)";
    return FBST_E_INVALID;
  }
  p.M = M;
  p.N = N;
  p.B = B;
  p.fc = band->fc;
  p.omega = band->omega;
  p.ts = band->ts;
  p.eps = 1.01;
  p.L = 2 * N;
  p.delta = 1e-5;
  p.prec = FBST_PREC_FP64;     // the paper's delta needs float64 (cond(A_b) ~ 2MN / delta)
  if (opt) {
    if (opt->eps != 0.0) p.eps = opt->eps;
    if (opt->L != 0) p.L = opt->L;
    p.delta = opt->delta;
    p.prec = opt->precision;
    p.flags = opt->flags;
  }
  if (!(p.eps > 0.0) || !std::isfinite(p.eps)) {
    *msg = "eps must be > 0";
    return FBST_E_INVALID;
  }
  if (p.L < 2 || (p.L % 2) != 0) {
    *msg = "L must be even and >= 2";
    return FBST_E_INVALID;
  }
  if (!(p.delta > 0.0) || !std::isfinite(p.delta)) {
    *msg = "delta must be > 0";
    return FBST_E_INVALID;
  }
  if (p.prec < FBST_PREC_FP32 || p.prec > FBST_PREC_FP16_SPLIT) {
    *msg = "unknown precision";
    return FBST_E_INVALID;
  }
  const double dflt = 1.0 / (2.0 * (p.fc + p.omega));
  if (!geom) {
    p.kind = FBST_LINE;
    p.mx = M;
    p.my = 1;
    p.dx = dflt;
  } else {
    p.kind = geom->kind;
    p.mx = geom->mx;
    p.my = geom->my;
    p.dx = geom->dx != 0.0 ? geom->dx : dflt;
    p.dy = geom->dy != 0.0 ? geom->dy : dflt;
    p.x0 = geom->x0;
    p.y0 = geom->y0;
    if (p.kind != FBST_LINE && p.kind != FBST_GRID && p.kind != FBST_ARBITRARY) {
      *msg = "unknown geometry kind";
      return FBST_E_INVALID;
    }
    if (p.kind == FBST_ARBITRARY) {
      if (!geom->px) {
        *msg = "an arbitrary array needs px (M element coordinates)";
        return FBST_E_INVALID;
      }
      p.px.assign(geom->px, geom->px + M);
      if (geom->py) p.py.assign(geom->py, geom->py + M);
      else p.py.assign(M, 0.0);
      for (int m = 0; m < M; ++m)
        if (!std::isfinite(p.px[m]) || !std::isfinite(p.py[m])) {
          *msg = "element coordinates must be finite";
          return FBST_E_INVALID;
        }
      p.mx = M;
      p.my = 1;
      p.dx = p.dy = p.x0 = p.y0 = 0.0;
    } else if (p.kind == FBST_LINE) {
      if (p.mx != M || p.my != 1) {
        *msg = "a line needs mx == M and my == 1";
        return FBST_E_INVALID;
      }
      p.dy = 0.0;
      p.y0 = 0.0;
    } else if (p.mx < 1 || p.my < 1 || 1LL * p.mx * p.my != M) {
      *msg = "a grid needs mx * my == M";
      return FBST_E_INVALID;
    }
    if (!std::isfinite(p.dx) || !std::isfinite(p.dy) || !std::isfinite(p.x0) || !std::isfinite(p.y0)) {
      *msg = "geometry values must be finite";
      return FBST_E_INVALID;
    }
  }
  const fbst_status gst = resolve_grid(&p, grid, msg);
  if (gst != FBST_OK) return gst;
  p.p1 = next_pow2(static_cast<long long>(p.N) + p.L - 1);
  p.p2x = next_pow2(static_cast<long long>(p.mx) + p.bu - 1);
  p.p2y = p.kind == FBST_GRID ? next_pow2(static_cast<long long>(p.my) + p.bv - 1) : 0;
  p.p3 = next_pow2(std::max(2LL * p.L - 1, static_cast<long long>(p.L) + p.N - 1));
  p.p2x = std::max(p.p2x, 32);
  if (p.kind == FBST_GRID) p.p2y = std::max(p.p2y, 32);
  if (p.kind == FBST_ARBITRARY) {
    // oversampled grids of at least twice the modes per axis; kernel width for
    // about float32 (8 points) or float64 (16 points) accuracy; shape
    // parameter beta = 0.98 pi (1 - 1/(2 sigma)) w for oversampling sigma
    p.p2x = std::max(next_pow2(2LL * p.bu), 32);
    p.p2y = p.bv > 1 ? std::max(next_pow2(2LL * p.bv), 32) : 0;
    p.nuw = (p.prec == FBST_PREC_FP64) ? 16 : 8;
    double sigma = static_cast<double>(p.p2x) / p.bu;
    if (p.p2y) sigma = std::min(sigma, static_cast<double>(p.p2y) / p.bv);
    p.nu_beta = 0.98 * kPi * (1.0 - 0.5 / sigma) * p.nuw;
    // LDS words of one frequency's grid (padded layout of the spread kernels)
    const double words = p.p2y ? static_cast<double>(p.p2x) * (p.p2y + 8) + 32.0
                               : static_cast<double>(p.p2x) * 17.0 / 16.0 + 32.0;
    const double grid_bytes = words * (p.prec == FBST_PREC_FP64 ? 16.0 : 8.0);
    if (grid_bytes > 144.0 * 1024) {
      *msg = "the oversampled grid of one frequency (" + std::to_string(p.p2x) + " x " +
             std::to_string(std::max(p.p2y, 1)) + ") exceeds 144 KiB of LDS";
      return FBST_E_UNSUPPORTED;
    }
  }
  p.p1 = std::max(p.p1, 32);
  p.p3 = std::max(p.p3, 32);
  if ((p.prec == FBST_PREC_BF16_SPLIT || p.prec == FBST_PREC_FP16_SPLIT) && p.p1 < 1024) {
    *msg = "the matrix-core stage 1a needs a time FFT of at least 1024 points (N + L - 1 > 512)";
    return FBST_E_UNSUPPORTED;
  }
  // Stage 1a in split-output form when it is smaller: the two output halves
  // need the chirp kernel over N + L/2 - 1 taps each, so two convolutions of
  // p1s points sharing one forward FFT replace one of p1 points (3 p1s
  // against 2 p1 transform points; p1s = p1 / 2 whenever L = 2N).
  if (!(p.flags & FBST_FLAG_NO_SPLIT) && p.prec != FBST_PREC_BF16_SPLIT &&
      p.prec != FBST_PREC_FP16_SPLIT) {
    const int ls = p.L / 2;
    const int ps = std::max(next_pow2(static_cast<long long>(p.N) + ls - 1), 32);
    if (2 * ps < 2 * p.p1 - ps) {       // 3 ps < 2 p1
      p.p1s = ps;
      p.ls1 = ls;
    }
  }
  if (p.flags & FBST_FLAG_DEVICE_GENERATORS) {
    if (p.flags & FBST_FLAG_HOST_ONLY) {
      *msg = "FBST_FLAG_DEVICE_GENERATORS needs a device plan (not FBST_FLAG_HOST_ONLY)";
      return FBST_E_INVALID;
    }
    if (p.L > 8192) {
      *msg = "the device generator solve holds L <= 8192 coefficients in LDS";
      return FBST_E_UNSUPPORTED;
    }
    if ((p.flags & FBST_FLAG_SUPERFAST_GENERATORS) && p.L > 4096) {
      *msg = "the device superfast generator solve holds transforms of 2L <= 8192 points in LDS "
             "(L <= 4096)";
      return FBST_E_UNSUPPORTED;
    }
  }
  if (p.flags & FBST_FLAG_STAGE2_REFINE) {
    if (p.prec == FBST_PREC_FP64 || p.prec == FBST_PREC_FP64_STAGE2) {
      *msg = "FBST_FLAG_STAGE2_REFINE refines a float32 stage 2 (not FBST_PREC_FP64 or "
             "FBST_PREC_FP64_STAGE2)";
      return FBST_E_UNSUPPORTED;
    }
    if (p.flags & FBST_FLAG_PRECOMPUTE) {
      *msg = "FBST_FLAG_STAGE2_REFINE and FBST_FLAG_PRECOMPUTE exclude each other";
      return FBST_E_UNSUPPORTED;
    }
  }
  if (p.flags & FBST_FLAG_PRECOMPUTE) {
    if (p.prec == FBST_PREC_FP64) {
      *msg = "the precomputed stage 2 takes complex64 data (any precision but FBST_PREC_FP64)";
      return FBST_E_UNSUPPORTED;
    }
    if (p.p3 > 8192) {
      *msg = "the precomputed stage 2 is built by the float64 stage-2 kernel (P3 <= 8192)";
      return FBST_E_UNSUPPORTED;
    }
    const double kbytes = 8.0 * p.L * p.B * p.N;
    if (kbytes > 16.0 * (1ULL << 30)) {
      *msg = "the precomputed stage 2 would hold " + std::to_string(kbytes / (1ULL << 30)) +
             " GiB of K (limit 16 GiB)";
      return FBST_E_UNSUPPORTED;
    }
  }
  // Stage 1 in float64 (FBST_PREC_FP64) holds one transform in LDS (8192
  // points; stage 1a in split-output form needs only p1s); stage 2 goes to
  // PMAX in every precision (in float64 above 8192 points each transform is
  // split into two halves in LDS).
  const int lim1 = (p.prec == FBST_PREC_FP64) ? 8192 : PMAX;
  const int p1_run = p.p1s ? p.p1s : p.p1;
  if (p1_run > lim1 || p.p1 > PMAX || p.p2x > lim1 || p.p2y > lim1 || p.p3 > PMAX) {
    *msg = "an FFT size exceeds what one workgroup holds in LDS for this precision";
    return FBST_E_UNSUPPORTED;
  }
  // Conditioning guard (Sec. V).  F_b^H F_b = sum_m D_m T D_m^H with T the
  // time Gram and D_m = diag(exp(j omega_l tau_{b,m})) unitary, so for every
  // beam and any geometry cond(A_b) <= 1 + M lambda_max(T) / delta.  A solve in
  // a precision of unit roundoff u can lose up to cond * u of relative
  // accuracy; plans whose bound exceeds 1e-2 (float32 stage 2: cond > 1.7e5,
  // about 1e-4 of measured beam error; float64: cond > 9e13) are refused
  // rather than built to return beams off by O(1).
  {
    const double lam = time_gram_lmax(p.N, p.L, p.eps);
    p.cond_bound = 1.0 + p.M * lam / p.delta;
    const bool s2_double = p.prec == FBST_PREC_FP64 || p.prec == FBST_PREC_FP64_STAGE2;
    const double u2 = s2_double ? 0x1.0p-53 : 0x1.0p-24;
    if (!(p.cond_bound * u2 <= 1e-2)) {
      char buf[320];
      std::snprintf(buf, sizeof buf,
                    "delta = %.3g is too small for a %s stage 2: cond(F^H F + delta I) can reach "
                    "%.3g (1 + M lambda_max(T)/delta), beyond the %.3g this precision holds; "
                    "raise delta towards the noise level (e.g. sigma^2 L) or use %s",
                    p.delta, s2_double ? "float64" : "float32", p.cond_bound, 1e-2 / u2,
                    s2_double ? "a larger delta" : "FBST_PREC_FP64");
      *msg = buf;
      return FBST_E_UNSUPPORTED;
    }
  }
  *out = p;
  return FBST_OK;
}

namespace {

// The tail of one beam's stage-2 tables from its Toeplitz column col (with
// delta) and generator x: refinement when cond(A) is large, the kept copies,
// and the Gohberg-Semencul spectra G1 = FFT(x), G2 = FFT(y~), both scaled by
// 1 / (P3 sqrt(x0)).
void finish_beam(const Params& p, int b, const zd* col, std::vector<zd>* xv, bool keep_gram_gen,
                 HostTables* t, std::vector<zd>* bufv) {
  const int L = p.L, P3 = p.p3;
  std::vector<zd>& x = *xv;
  std::vector<zd>& buf = *bufv;
  // refine the generators when cond(A) ~ 2MN/delta makes their float64
  // forward error visible (above ~1e6)
  const bool refine = 2.0 * p.M * p.N / p.delta > 1e6;
  if (keep_gram_gen) std::copy(col, col + L, t->gram.begin() + static_cast<size_t>(b) * L);
  if (refine) {
    // the superfast solve's forward error grows faster with cond(A) than
    // Levinson's: up to three steps instead of one
    const int steps = (p.flags & FBST_FLAG_SUPERFAST_GENERATORS) ? 3 : 1;
    for (int s = 0; s < steps; ++s) refine_generator(col, L, P3, &x);
  }
  if (keep_gram_gen) std::copy(x.begin(), x.end(), t->gen.begin() + static_cast<size_t>(b) * L);
  const double scale = 1.0 / (P3 * std::sqrt(x[0].real()));
  std::fill(buf.begin(), buf.end(), zd());
  std::copy(x.begin(), x.end(), buf.begin());
  fft64(buf.data(), P3, -1);
  for (int i = 0; i < P3; ++i) t->G1[static_cast<size_t>(b) * P3 + i] = buf[i] * scale;
  // y~ = (0, conj x_{L-1}, ..., conj x_1)
  std::fill(buf.begin(), buf.end(), zd());
  for (int i = 1; i < L; ++i) buf[i] = std::conj(x[L - i]);
  fft64(buf.data(), P3, -1);
  for (int i = 0; i < P3; ++i) t->G2[static_cast<size_t>(b) * P3 + i] = buf[i] * scale;
  if (p.flags & FBST_FLAG_STAGE2_REFINE) {
    // A_b as a circulant of P3 points: first column c_0 .. c_{L-1}, zeros, then
    // conj(c_{L-1}) .. conj(c_1) (A_b Hermitian), so A_b v = first L of the
    // circular convolution with v zero-padded; spectrum divided by P3 for the
    // unscaled inverse transform of the kernel
    std::fill(buf.begin(), buf.end(), zd());
    for (int i = 0; i < L; ++i) buf[i] = col[i];
    for (int i = 1; i < L; ++i) buf[P3 - i] = std::conj(col[i]);
    fft64(buf.data(), P3, -1);
    for (int i = 0; i < P3; ++i) t->CA[static_cast<size_t>(b) * P3 + i] = buf[i] / static_cast<double>(P3);
  }
}

}  // namespace

namespace {

struct HostSync {
  void operator()() const {}
  void wave() const {}
};

}  // namespace

std::vector<zd> superfast_twiddles(int L) {
  const int PM = superfast::max_fft(L);
  std::vector<zd> tw(PM / 2);
  for (int k = 0; k < PM / 2; ++k) tw[k] = cis(-2.0 * kPi * k / PM);
  return tw;
}

bool superfast_first_column(const zd* col, int L, zd* x) {
  const std::vector<zd> tw = superfast_twiddles(L);
  std::vector<zd> scratch(superfast::scratch_elems(L)), lds(superfast::lds_elems(L));
  using Z = superfast::z;
  const superfast::Ctx c{0, 1, reinterpret_cast<const Z*>(tw.data()), superfast::max_fft(L)};
  return superfast::generator(reinterpret_cast<const Z*>(col), reinterpret_cast<Z*>(x), L,
                              reinterpret_cast<Z*>(scratch.data()), reinterpret_cast<Z*>(lds.data()),
                              c, HostSync{});
}

fbst_status finish_generators(const Params& p, const std::vector<zd>& x, bool keep_gram_gen,
                              HostTables* t) {
  const int L = p.L, B = p.B;
  if (t->cols.size() != static_cast<size_t>(B) * L || x.size() != t->cols.size())
    return FBST_E_INVALID;
  parallel_for(B, 1LL * B * p.p3 * 64, [&](int b0, int b1) {
    std::vector<zd> xb(L), buf(p.p3);
    for (int b = b0; b < b1; ++b) {
      std::copy(x.begin() + static_cast<size_t>(b) * L, x.begin() + static_cast<size_t>(b + 1) * L,
                xb.begin());
      finish_beam(p, b, t->cols.data() + static_cast<size_t>(b) * L, &xb, keep_gram_gen, t, &buf);
    }
  });
  t->cols.clear();
  t->cols.shrink_to_fit();
  return FBST_OK;
}

fbst_status build_tables(const Params& p, bool keep_gram_gen, HostTables* t, std::string* msg) {
  const int N = p.N, L = p.L, B = p.B;
  const double lp0 = 1.0 - 0.5 * L;             // l' of the first basis frequency
  // kappa = 2 pi eps / L rad per sample and per unit of l'; phases of the
  // chirps are (kappa/2) k^2 = pi * (eps / L) * k^2.
  const double c_pi = p.eps / L;

  // --- stage 1a: Yhat[i] = post1[i] sum_n (x[n] pre1[n]) h1[i - n] -------------
  t->pre1.resize(N);
  for (int n = 0; n < N; ++n) t->pre1[n] = cispi(-c_pi * static_cast<double>(1LL * n * n));
  // h1[s] = exp(+j (kappa/2) (s + lp0)^2) for s in [-(N-1), L-1]
  if (p.p1s) {
    // output half h covers i = h ls1 + i', i' < len_h: kernel h1[s + h ls1], s in [-(N-1), len_h - 1]
    const long long ls = p.ls1;
    t->H1a = kernel_spectrum_int(p.p1s, -(N - 1), ls - 1, static_cast<long long>(lp0), c_pi);
    t->H1b = kernel_spectrum_int(p.p1s, -(N - 1), (L - ls) - 1, static_cast<long long>(lp0) + ls,
                                 c_pi);
  } else {
    t->H1 = kernel_spectrum_int(p.p1, -(N - 1), L - 1, static_cast<long long>(lp0), c_pi);
  }
  t->post1.resize(L);
  for (int i = 0; i < L; ++i) {
    const long long q = static_cast<long long>(i + lp0);
    t->post1[i] = cispi(-c_pi * static_cast<double>(q * q));
  }

  // --- stage 1b: spatial chirp-z per axis ------------------------------------
  if (p.kind == FBST_ARBITRARY) {
    build_nonuniform(p, t);
  } else {
    build_axis(p, p.mx, p.bu, p.x0, p.dx / p.ts, p.u0, p.du, p.p2x, &t->ax);
    if (p.kind == FBST_GRID) build_axis(p, p.my, p.bv, p.y0, p.dy / p.ts, p.v0, p.dv, p.p2y, &t->ay);
  }

  // --- beams ---------------------------------------------------------------
  t->u.resize(B);
  t->v.resize(B);
  for (int a = 0; a < p.bu; ++a)
    for (int c = 0; c < p.bv; ++c) {
      t->u[a * p.bv + c] = p.u0 + a * p.du;
      t->v[a * p.bv + c] = (p.kind != FBST_LINE) ? p.v0 + c * p.dv : 0.0;
    }

  // --- stage 2 F_u chirp-z: b[n] = post3[n] sum_i (beta[i] pre3[i]) h3[n - i] -----
  t->pre3.resize(L);
  for (int i = 0; i < L; ++i) {
    const long long q = static_cast<long long>(i + lp0);
    t->pre3[i] = cispi(c_pi * static_cast<double>(q * q));
  }
  // h3[s] = exp(-j (kappa/2) (s - lp0)^2) for s in [-(L-1), N-1]
  t->H3 = kernel_spectrum_int(p.p3, -(L - 1), N - 1, -static_cast<long long>(lp0), -c_pi);
  t->post3.resize(N);
  for (int n = 0; n < N; ++n) t->post3[n] = cispi(c_pi * static_cast<double>(1LL * n * n));

  // --- stage 2 Toeplitz generators (Sec. V) -----------------------------------
  // c_b(d) = [sum_n e^{-j kd n}] [sum_k e^{j kd u px_k}] [sum_k2 e^{j kd v py_k2}],
  // kd = 2 pi eps d / L (per sample), px, py in samples; A_b = toeplitz(c_b) + delta I.
  const int P3 = p.p3;
  t->G1.assign(static_cast<size_t>(B) * P3, zd());
  t->G2.assign(static_cast<size_t>(B) * P3, zd());
  if (p.flags & FBST_FLAG_STAGE2_REFINE) t->CA.assign(static_cast<size_t>(B) * P3, zd());
  if (keep_gram_gen) {
    t->gram.assign(static_cast<size_t>(B) * L, zd());
    t->gen.assign(static_cast<size_t>(B) * L, zd());
  } else {
    t->gram.clear();
    t->gen.clear();
  }
  // In a frame centred in time and on the array, c_b(d) = exp(-j kd s_b) r_b(d)
  // with kd = 2 pi eps d / L, s_b = (N-1)/2 - u dx (x0 + (mx-1)/2) - v dy (y0 + (my-1)/2)
  // (samples) and r_b(d) = D_N(kd) D_mx(kd u dx) D_my(kd v dy), D_K(y) =
  // sin(K y / 2) / sin(y / 2) real and even.  So A_b = D (R_b + delta I) D^H with
  // D = diag(exp(-j kd_l s_b)) and R_b real symmetric Toeplitz depending on
  // (|u|, |v|) only: x_b = A_b^{-1} e_0 = D (R_b + delta I)^{-1} e_0, one real
  // Levinson recursion per distinct (|u|, |v|).
  const double dxs = p.dx / p.ts, dys = p.dy / p.ts;
  auto dirichlet = [](int K, double y) {
    const double s = std::sin(0.5 * y);
    return s == 0.0 ? static_cast<double>(K) : std::sin(0.5 * K * y) / s;
  };
  std::vector<double> rt(L);
  for (int d = 0; d < L; ++d) rt[d] = dirichlet(N, 2.0 * kPi * p.eps * d / L);
  std::vector<int> key_of(B);
  std::vector<std::pair<double, double>> keys;
  if (p.kind != FBST_ARBITRARY) {
    std::vector<std::pair<std::pair<double, double>, int>> seen;
    for (int b = 0; b < B; ++b) {
      const std::pair<double, double> k(std::fabs(t->u[b]), std::fabs(t->v[b]));
      int idx = -1;
      for (const auto& e : seen)
        if (e.first == k) { idx = e.second; break; }
      if (idx < 0) {
        idx = static_cast<int>(keys.size());
        keys.push_back(k);
        seen.push_back({k, idx});
      }
      key_of[b] = idx;
    }
  }
  const int K = static_cast<int>(keys.size());
  // generators solved on the device (FBST_FLAG_DEVICE_GENERATORS): keep the
  // columns only; finish_generators completes the tables
  const bool device = (p.flags & FBST_FLAG_DEVICE_GENERATORS) != 0;
  const bool superfast = (p.flags & FBST_FLAG_SUPERFAST_GENERATORS) != 0;
  if (device) t->cols.assign(static_cast<size_t>(B) * L, zd());
  std::vector<std::vector<double>> rcol(K), xr(K);
  std::atomic<bool> ok{true};
  std::mutex fail_mu;
  std::string fail;
  auto real_work = [&](int k0, int k1) {
    for (int k = k0; k < k1 && ok.load(); ++k) {
      std::vector<double>& r = rcol[k];
      r.resize(L);
      const double au = keys[k].first, av = keys[k].second;
      for (int d = 0; d < L; ++d) {
        const double kd = 2.0 * kPi * p.eps * d / L;
        double v = rt[d] * dirichlet(p.mx, kd * au * dxs);
        if (p.kind == FBST_GRID) v *= dirichlet(p.my, kd * av * dys);
        r[d] = v;
      }
      r[0] += p.delta;
      if (device) continue;
      xr[k].resize(L);
      bool solved;
      if (superfast) {
        std::vector<zd> cz(r.begin(), r.end()), xz(L);
        solved = superfast_first_column(cz.data(), L, xz.data());
        for (int d = 0; d < L; ++d) xr[k][d] = xz[d].real();
      } else {
        solved = levinson_real(r.data(), L, xr[k].data());
      }
      if (!solved) {
        std::lock_guard<std::mutex> lk(fail_mu);
        ok = false;
        fail = "Toeplitz system not positive definite in float64 (delta too small?)";
      }
    }
  };
  auto work = [&](int b0, int b1) {
    std::vector<zd> col(L), x(L), buf(P3);
    for (int b = b0; b < b1 && ok.load(); ++b) {
      const double ub = t->u[b], vb = t->v[b];
      if (p.kind == FBST_ARBITRARY) {
        // no closed form: the sensor sum directly, then complex Levinson
        for (int d = 0; d < L; ++d) {
          const double kd = 2.0 * kPi * p.eps * d / L;
          col[d] = geometric_sum(N, 0.0, -kd) * sensor_sum(p, kd * ub, kd * vb);
        }
        col[0] = zd(col[0].real() + p.delta, 0.0);
        if (!device && !(superfast ? superfast_first_column(col.data(), L, x.data())
                                   : levinson_first_column(col.data(), L, x.data()))) {
          std::lock_guard<std::mutex> lk(fail_mu);
          ok = false;
          fail = "Toeplitz system not positive definite in float64 (delta too small?)";
          break;
        }
      } else {
        const double sb = 0.5 * (N - 1) - ub * dxs * (p.x0 + 0.5 * (p.mx - 1)) -
                          ((p.kind == FBST_GRID) ? vb * dys * (p.y0 + 0.5 * (p.my - 1)) : 0.0);
        const std::vector<double>& r = rcol[key_of[b]];
        for (int d = 0; d < L; ++d) col[d] = cis(-2.0 * kPi * p.eps * d / L * sb) * r[d];
        col[0] = zd(r[0], 0.0);
        if (!device) {
          const std::vector<double>& xk = xr[key_of[b]];
          for (int d = 0; d < L; ++d) x[d] = cis(-2.0 * kPi * p.eps * d / L * sb) * xk[d];
          x[0] = zd(xk[0], 0.0);
        }
      }
      if (device) {
        std::copy(col.begin(), col.end(), t->cols.begin() + static_cast<size_t>(b) * L);
        continue;
      }
      finish_beam(p, b, col.data(), &x, keep_gram_gen, t, &buf);
    }
  };
  parallel_for(K, 1LL * K * L * L, real_work);
  if (!ok) {
    *msg = fail;
    return FBST_E_INVALID;
  }
  parallel_for(B, 1LL * B * P3 * 64 + (p.kind == FBST_ARBITRARY ? 1LL * B * L * (L + p.M) * 8 : 0),
               work);
  if (!ok) {
    *msg = fail;
    return FBST_E_INVALID;
  }
  return FBST_OK;
}

// --- a new beam grid for an existing plan (line or planar grid) -------------
// The tables that depend on the beam directions: the stage-1b chirps of each
// axis, the beams' (u, v), and the Toeplitz first columns [B][L] (with delta)
// of the new beams in the closed form of build_tables (a frame centred in
// time and on the array: c_b(d) = exp(-j kd s_b) r_b(d)); the generators and
// their spectra are left to the caller.
fbst_status build_steer_tables(const Params& p, HostTables* t, SteerKeys* k, bool cols,
                               std::string* msg) {
  if (p.kind == FBST_ARBITRARY) {
    *msg = "a new beam grid is supported for lines and uniform grids";
    return FBST_E_UNSUPPORTED;
  }
  const int N = p.N, L = p.L, B = p.B;
  build_axis(p, p.mx, p.bu, p.x0, p.dx / p.ts, p.u0, p.du, p.p2x, &t->ax);
  if (p.kind == FBST_GRID) build_axis(p, p.my, p.bv, p.y0, p.dy / p.ts, p.v0, p.dv, p.p2y, &t->ay);
  t->u.resize(B);
  t->v.resize(B);
  for (int a = 0; a < p.bu; ++a)
    for (int c = 0; c < p.bv; ++c) {
      t->u[a * p.bv + c] = p.u0 + a * p.du;
      t->v[a * p.bv + c] = (p.kind != FBST_LINE) ? p.v0 + c * p.dv : 0.0;
    }
  const double dxs = p.dx / p.ts, dys = p.dy / p.ts;
  auto dirichlet = [](int K, double y) {
    const double s = std::sin(0.5 * y);
    return s == 0.0 ? static_cast<double>(K) : std::sin(0.5 * K * y) / s;
  };
  std::vector<double> rt(L);
  for (int d = 0; d < L; ++d) rt[d] = dirichlet(N, 2.0 * kPi * p.eps * d / L);
  // distinct (|u|, |v|), as build_tables keys its real solves
  std::vector<std::pair<double, double>> keys;
  k->key.assign(B, 0);
  k->s.assign(B, 0.0);
  for (int b = 0; b < B; ++b) {
    const std::pair<double, double> kv(std::fabs(t->u[b]), std::fabs(t->v[b]));
    int idx = -1;
    for (size_t i = 0; i < keys.size(); ++i)
      if (keys[i] == kv) { idx = static_cast<int>(i); break; }
    if (idx < 0) {
      idx = static_cast<int>(keys.size());
      keys.push_back(kv);
    }
    k->key[b] = idx;
    k->s[b] = 0.5 * (N - 1) - t->u[b] * dxs * (p.x0 + 0.5 * (p.mx - 1)) -
              ((p.kind == FBST_GRID) ? t->v[b] * dys * (p.y0 + 0.5 * (p.my - 1)) : 0.0);
  }
  const int K = static_cast<int>(keys.size());
  k->rcols.assign(static_cast<size_t>(K) * L, zd());
  parallel_for(K, 1LL * K * L * 64, [&](int q0, int q1) {
    for (int q = q0; q < q1; ++q) {
      zd* r = k->rcols.data() + static_cast<size_t>(q) * L;
      for (int d = 0; d < L; ++d) {
        const double kd = 2.0 * kPi * p.eps * d / L;
        double v = rt[d] * dirichlet(p.mx, kd * keys[q].first * dxs);
        if (p.kind == FBST_GRID) v *= dirichlet(p.my, kd * keys[q].second * dys);
        r[d] = zd(v, 0.0);
      }
      r[0] += p.delta;
    }
  });
  if (!cols) {
    t->cols.clear();
    return FBST_OK;
  }
  // the complex columns of each beam (for the host refinement)
  t->cols.assign(static_cast<size_t>(B) * L, zd());
  parallel_for(B, 1LL * B * L * 16, [&](int b0, int b1) {
    for (int b = b0; b < b1; ++b) {
      const zd* r = k->rcols.data() + static_cast<size_t>(k->key[b]) * L;
      zd* col = t->cols.data() + static_cast<size_t>(b) * L;
      for (int d = 0; d < L; ++d) col[d] = cis(-2.0 * kPi * p.eps * d / L * k->s[b]) * r[d].real();
      col[0] = zd(r[0].real(), 0.0);
    }
  });
  (void)msg;
  return FBST_OK;
}

// --- beams at arbitrary directions (Sec. VIII, off-grid angles) ---------------
// For directions (ud, vd): K [l][d][n] = (F_u A_d^{-1})[n][l] (row n of
// F_u A_d^{-1} is conj(A_d^{-1} conj(row n of F_u)), A_d Hermitian; applied with
// the Gohberg-Semencul form of the refined generator of A_d), and the
// projection phases E [d][m][l] = exp(j a_l tau_{d,m}); float64.
fbst_status build_direction_tables(const Params& p, const std::vector<double>& ud,
                                   const std::vector<double>& vd, std::vector<zd>* K,
                                   std::vector<zd>* E, std::string* msg) {
  const int L = p.L, N = p.N, M = p.M, D = static_cast<int>(ud.size());
  const int PG = next_pow2(2LL * L);
  const double lp0 = 1.0 - 0.5 * L;
  const double kap = 2.0 * kPi * p.eps / L;
  auto a_of = [&](int l) { return 2.0 * kPi * p.fc * p.ts + kap * (l + lp0); };
  K->assign(static_cast<size_t>(L) * D * N, zd());
  if (E) E->assign(static_cast<size_t>(D) * M * L, zd());
  for (int di = 0; di < D; ++di) {
    // A_d = F_d^H F_d + delta I: c(d) = [sum_n e^{-j kappa d n}][sum_m e^{j kappa d tau_m}] + delta
    std::vector<zd> col(L), x(L);
    for (int d = 0; d < L; ++d) {
      const double kd = kap * d;
      col[d] = geometric_sum(N, 0.0, -kd) * sensor_sum(p, kd * ud[di], kd * vd[di]);
    }
    col[0] += p.delta;
    if (!levinson_first_column(col.data(), L, x.data())) {
      *msg = "direction Toeplitz system not positive definite in float64";
      return FBST_E_INVALID;
    }
    refine_generator(col.data(), L, PG, &x);
    parallel_for(N, 1LL * N * PG * 40, [&](int n0, int n1) {
      std::vector<zd> row(L), g;
      for (int n = n0; n < n1; ++n) {
        // row n of F_u: exp(j omega_l t_n), omega_l t_n = kappa l' n (eq. bhatls)
        for (int l = 0; l < L; ++l) row[l] = std::conj(cis(kap * (l + lp0) * n));
        gs_apply(x, row, L, PG, &g);
        for (int l = 0; l < L; ++l) (*K)[(static_cast<size_t>(l) * D + di) * N + n] = std::conj(g[l]);
      }
    });
    for (int m = 0; E && m < M; ++m) {
      const double tau = ud[di] * pos_x(p, m) + vd[di] * pos_y(p, m);
      for (int l = 0; l < L; ++l) (*E)[(static_cast<size_t>(di) * M + m) * L + l] = cis(a_of(l) * tau);
    }
  }
  return FBST_OK;
}

// --- beamspace nulling tables (Sec. VIII, eq. interfer_beam_space) ------------
// G [q L + k][b][n] = (G_{b,q})[n][k] with G_{b,q} = F_b^H F_q A_q^{-1}, for the
// interferer directions (uq, vq) (on or off the grid) and every beam b of the
// grid of p.  F_b^H F_q is the
// product of a time sum and a sensor sum (closed forms); row n of G_{b,q} is
// conj(A_q^{-1} conj(row n of F_b^H F_q)) (A_q Hermitian), applied with the
// Gohberg-Semencul form of the refined generator of A_q, all in float64.
// G maps w_q to the part of w_b that interferer q's fit contributes; its
// entries are O(1) (for b = q, G = I - delta A_q^{-1}), so storing it in
// float32 costs only float32 rounding of the data.
fbst_status build_null_tables(const Params& p, const std::vector<double>& uq,
                              const std::vector<double>& vq, std::vector<zd>* G,
                              std::vector<zd>* E, std::string* msg) {
  const int L = p.L, N = p.N, B = p.B, P = static_cast<int>(uq.size());
  const int PG = next_pow2(2LL * L);
  const double lp0 = 1.0 - 0.5 * L;
  const double kap = 2.0 * kPi * p.eps / L;                     // rad per sample per unit l'
  auto beam_u = [&](int b) { return p.u0 + (b / p.bv) * p.du; };
  auto beam_v = [&](int b) { return p.kind != FBST_LINE ? p.v0 + (b % p.bv) * p.dv : 0.0; };
  // time factor sum_n exp(-j kappa d n), d = l - k in (-L, L)
  std::vector<zd> tf(2 * L - 1);
  for (int d = -(L - 1); d <= L - 1; ++d) tf[d + L - 1] = geometric_sum(N, 0.0, -kap * d);
  // sensor factor sum_m exp(j (a_n tau_{b,m} - a_k tau_{q,m})) between direction
  // (ub, vb) and (uq, vq), tau in samples, a_l = 2 pi (f_c T_s) + kappa l'
  // (rad per sample of delay), separable per axis
  auto sensor2 = [&](double an, double ak, double ub, double vb, double u2, double v2) {
    return sensor_sum(p, an * ub - ak * u2, an * vb - ak * v2);
  };
  auto a_of = [&](int l) { return 2.0 * kPi * p.fc * p.ts + kap * (l + lp0); };
  // generators x_q = A_q^{-1} e_0 of A_q = F_q^H F_q + delta I (Sec. V), refined
  std::vector<std::vector<zd>> xq(P);
  for (int qi = 0; qi < P; ++qi) {
    std::vector<zd> col(L);
    xq[qi].resize(L);
    for (int d = 0; d < L; ++d)
      col[d] = tf[d + L - 1] * sensor2(a_of(d), a_of(0), uq[qi], vq[qi], uq[qi], vq[qi]);
    col[0] += p.delta;
    if (!levinson_first_column(col.data(), L, xq[qi].data())) {
      *msg = "interferer Toeplitz system not positive definite in float64";
      return FBST_E_INVALID;
    }
    refine_generator(col.data(), L, PG, &xq[qi]);
  }
  G->assign(static_cast<size_t>(P) * L * B * L, zd());
  parallel_for(B, 1LL * B * P * L * PG * 40, [&](int b0, int b1) {
    std::vector<zd> row(L), g;
    for (int b = b0; b < b1; ++b)
      for (int qi = 0; qi < P; ++qi)
        for (int n = 0; n < L; ++n) {
          const double an = a_of(n);
          for (int k = 0; k < L; ++k)
            row[k] = std::conj(tf[n - k + L - 1] *
                               sensor2(an, a_of(k), beam_u(b), beam_v(b), uq[qi], vq[qi]));
          gs_apply(xq[qi], row, L, PG, &g);
          for (int k = 0; k < L; ++k)
            (*G)[((static_cast<size_t>(qi) * L + k) * B + b) * L + n] = std::conj(g[k]);
        }
  });
  // projection phases of the interferer directions, E [q][m][l] = exp(j a_l tau_{q,m}),
  // m = k * my + k2 (so that w_q[l] = sum_m Yhat[m][l] E[q][m][l], Sec. IV)
  if (E) {
    const int M = p.M;
    E->assign(static_cast<size_t>(P) * M * L, zd());
    for (int qi = 0; qi < P; ++qi)
      for (int m = 0; m < M; ++m) {
        const double tau = uq[qi] * pos_x(p, m) + vq[qi] * pos_y(p, m);
        for (int l = 0; l < L; ++l)
          (*E)[(static_cast<size_t>(qi) * M + m) * L + l] = cis(a_of(l) * tau);
      }
  }
  return FBST_OK;
}

// Off-grid beams by spline interpolation (Sec. VIII).  In the grid index
// s = (u - u0) / du the beams sit at the integers, and an affine change of
// variable maps a cubic spline to a cubic spline with the same end
// conditions, so the weights follow from unit-spaced nodes 0..7.  With
// moments M_k = S''(k), the spline through node values y is
//   S(x) = M_k a^3 / 6 + M_{k+1} b^3 / 6 + (y_k - M_k / 6) a + (y_{k+1} - M_{k+1} / 6) b,
//   a = k + 1 - x, b = x - k on [k, k + 1],
// where the interior nodes give M_{k-1} + 4 M_k + M_{k+1} = 6 (y_{k-1} - 2 y_k + y_{k+1})
// and the not-a-knot ends M_0 - 2 M_1 + M_2 = 0 = M_5 - 2 M_6 + M_7 (equal
// third derivatives on the first two and on the last two intervals).  The
// weight of node i is the spline through the unit vector e_i.
namespace {
void spline_unit_weights(double x, double* w) {
  constexpr int n = INTERP_TAPS;
  for (int i = 0; i < n; ++i) {
    double A[n][n + 1] = {};
    A[0][0] = 1.0; A[0][1] = -2.0; A[0][2] = 1.0;
    A[n - 1][n - 3] = 1.0; A[n - 1][n - 2] = -2.0; A[n - 1][n - 1] = 1.0;
    for (int k = 1; k < n - 1; ++k) {
      A[k][k - 1] = 1.0; A[k][k] = 4.0; A[k][k + 1] = 1.0;
      A[k][n] = 6.0 * ((k - 1 == i) - 2.0 * (k == i) + (k + 1 == i));
    }
    // Gaussian elimination with partial pivoting, then back substitution
    for (int c = 0; c < n; ++c) {
      int piv = c;
      for (int r = c + 1; r < n; ++r)
        if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
      if (piv != c)
        for (int k = 0; k <= n; ++k) std::swap(A[c][k], A[piv][k]);
      for (int r = c + 1; r < n; ++r) {
        const double f = A[r][c] / A[c][c];
        for (int k = c; k <= n; ++k) A[r][k] -= f * A[c][k];
      }
    }
    double Mo[n];
    for (int r = n - 1; r >= 0; --r) {
      double acc = A[r][n];
      for (int k = r + 1; k < n; ++k) acc -= A[r][k] * Mo[k];
      Mo[r] = acc / A[r][r];
    }
    int k = static_cast<int>(std::floor(x));
    if (k < 0) k = 0;
    if (k > n - 2) k = n - 2;
    const double a = k + 1 - x, b = x - k;
    const double yk = (k == i), yk1 = (k + 1 == i);
    w[i] = Mo[k] * a * a * a / 6.0 + Mo[k + 1] * b * b * b / 6.0 + (yk - Mo[k] / 6.0) * a +
           (yk1 - Mo[k + 1] / 6.0) * b;
  }
}
}  // namespace

fbst_status build_interp_table(const Params& p, const std::vector<double>& ud,
                               const std::vector<double>& vd, std::vector<int>* first,
                               std::vector<double>* w, std::string* msg,
                               std::vector<double>* frac) {
  const bool plane = p.bv > 1;
  if (p.bu < INTERP_TAPS || p.du == 0.0 || (plane && (p.bv < INTERP_TAPS || p.dv == 0.0))) {
    *msg = "spline interpolation needs at least 8 distinct grid beams along each axis";
    return FBST_E_UNSUPPORTED;
  }
  // window and weights along one axis with n beams at x0 + k dx
  auto axis = [](double x, double x0, double dx, int n, int* f, double* ww, double* fr) {
    const double last = n - 1;
    // position on the grid, x = x0 + s dx; the direction itself, not the
    // clamped s, sets the offset from the window (a hair outside the ends)
    const double s_raw = (x - x0) / dx;
    const double tol = 1e-9 * n;
    if (!(s_raw >= -tol && s_raw <= last + tol)) return false;
    const double s = std::min(std::max(s_raw, 0.0), last);
    const int j = std::min(static_cast<int>(std::floor(s)), n - 1);   // x_j <= x < x_{j+1}
    const int j0 = std::min(std::max(j - (INTERP_TAPS / 2 - 1), 0), n - INTERP_TAPS);
    *f = j0;
    spline_unit_weights(s - j0, ww);
    *fr = s_raw - j0;
    return true;
  };
  const size_t D = ud.size();
  first->assign(2 * D, 0);
  w->assign(2 * D * INTERP_TAPS, 0.0);
  std::vector<double> fr(2 * D, 0.0);
  for (size_t d = 0; d < D; ++d) {
    int* f = first->data() + 2 * d;
    double* ww = w->data() + 2 * d * INTERP_TAPS;
    bool ok = axis(ud[d], p.u0, p.du, p.bu, f, ww, &fr[2 * d]);
    if (plane) ok = ok && axis(vd[d], p.v0, p.dv, p.bv, f + 1, ww + INTERP_TAPS, &fr[2 * d + 1]);
    else ww[INTERP_TAPS] = 1.0;                 // one beam along v, weight 1
    if (!ok) {
      *msg = "interpolation directions must lie within the beam grid (no extrapolation)";
      return FBST_E_INVALID;
    }
  }
  if (frac) *frac = std::move(fr);
  return FBST_OK;
}

void reference_phase_rates(const Params& p, std::vector<double>* theta) {
  const int L = p.L;
  const double lp0 = 1.0 - 0.5 * L;
  const double kap = 2.0 * kPi * p.eps / L;
  double xmin = 0, xmax = 0, ymin = 0, ymax = 0;
  for (int m = 0; m < p.M; ++m) {
    const double x = pos_x(p, m), y = pos_y(p, m);
    if (m == 0 || x < xmin) xmin = x;
    if (m == 0 || x > xmax) xmax = x;
    if (m == 0 || y < ymin) ymin = y;
    if (m == 0 || y > ymax) ymax = y;
  }
  const double cx = 0.5 * (xmin + xmax), cy = 0.5 * (ymin + ymax);
  theta->assign(2 * static_cast<size_t>(L), 0.0);
  for (int l = 0; l < L; ++l) {
    // a_l = 2 pi f_c T_s + kappa l' radians per sample of delay (Sec. IV)
    const double a = 2.0 * kPi * p.fc * p.ts + kap * (l + lp0);
    (*theta)[l] = a * cx * p.du;
    (*theta)[L + l] = (p.bv > 1) ? a * cy * p.dv : 0.0;
  }
}

}  // namespace fbst
