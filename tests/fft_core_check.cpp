// Host check of the merged radix-16 butterflies of csrc/fft_lds.h: a twiddled
// Stockham pass, DFT_16 of x_r w^{r k} with w = exp(-2 pi j / (16 NS)), done
// by dft16_m from the merged factors as fft_lds.h defines them (psi^2, psi,
// -j psi, then om^2, om, -j om for k1 = 0..3, psi = w^{4k}, om = w^k
// w_16^{k1}, each as (Re f, Im f / Re f) with |Re f| >= 2^-40), against the
// direct sum in double, both directions.  Prints the largest relative errors;
// exit status 0 when they are within 4e-7 (float) and 2e-12 (double).
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>

#include "fft_lds.h"

using namespace fbst;
using zd = std::complex<double>;

namespace {

const double kPi = 3.141592653589793238462643383279502884;

zd unit(long long m, long long D) {   // exp(-2 pi j m / D)
  const double a = 2.0 * kPi * static_cast<double>(((m % D) + D) % D) / static_cast<double>(D);
  return zd(std::cos(a), -std::sin(a));
}

zd factor(long long m, long long D) {
  const zd f = unit(m, D);
  double c = f.real();
  const double lim = std::ldexp(1.0, -40);
  if (std::fabs(c) < lim) c = std::signbit(c) ? -lim : lim;
  return zd(c, f.imag() / c);
}

template <int DIR, typename T>
void check(int NS, int k, std::mt19937& g, double& e_merged) {
  const long long D = 16LL * NS, q = 4LL * NS;
  std::normal_distribution<double> nd;
  zd x[16];
  for (auto& z : x) z = zd(nd(g), nd(g));
  zd ref[16];
  double nrm = 0.0;
  for (int kp = 0; kp < 16; ++kp) {
    zd s = 0.0;
    for (int r = 0; r < 16; ++r) {
      const zd w = unit(1LL * r * k + 1LL * r * kp * NS, D);
      s += x[r] * (DIR < 0 ? w : std::conj(w));
    }
    ref[kp] = s;
    nrm += std::norm(s);
  }
  auto err = [&](const cx<T>(&v)[16]) {
    double e = 0.0;
    for (int kp = 0; kp < 16; ++kp) e += std::norm(zd(v[kp].re, v[kp].im) - ref[kp]);
    return std::sqrt(e / nrm);
  };
  // merged factors
  cx<T> f[15];
  auto put = [&](int i, long long m) {
    const zd z = factor(m, D);
    f[i] = cx<T>{static_cast<T>(z.real()), static_cast<T>(z.imag())};
  };
  put(0, 8LL * k);
  put(1, 4LL * k);
  put(2, 4LL * k + q);
  for (int k1 = 0; k1 < 4; ++k1) {
    const long long o = k + 1LL * NS * k1;
    put(3 + 3 * k1, 2 * o);
    put(4 + 3 * k1, o);
    put(5 + 3 * k1, o + q);
  }
  cx<T> b[16];
  for (int r = 0; r < 16; ++r) b[r] = cx<T>{static_cast<T>(x[r].real()), static_cast<T>(x[r].imag())};
  dft16_m<DIR>(b, [&](int i) { return f[i]; });
  e_merged = std::max(e_merged, err(b));
}

}  // namespace

int main() {
  std::mt19937 g(20261203);
  double mf = 0, md = 0;
  for (int NS : {16, 64, 256, 1024, 4096}) {
    const int step = NS <= 256 ? 1 : 13;
    for (int k = 0; k < NS; k += step) {
      check<-1, float>(NS, k, g, mf);
      check<+1, float>(NS, k, g, mf);
      check<-1, double>(NS, k, g, md);
      check<+1, double>(NS, k, g, md);
    }
  }
  std::printf("merged radix-16 pass: float %.3e, double %.3e\n", mf, md);
  return (mf < 4e-7 && md < 2e-12) ? 0 : 1;
}
