// Spectra of the Gohberg-Semencul factors of stage 2 (Sec. V) on the GPU,
// from the generators x_b = A_b^{-1} e_0 [B][L] (complex128):
//   G1_b = FFT_P(x_b) s_b,  G2_b = FFT_P(y~_b) s_b,  s_b = 1 / (P sqrt(x_b[0])),
//   y~_b = (0, conj x_b[L-1], ..., conj x_b[1]),
// both zero-padded to P points, computed in float64 and stored in the stage-2
// type.  With key given, x holds the generators of real centred systems
// [K][L] and x_b[d] = x[key[b]][d] exp(-j 2 pi eps d s[b] / L) (the phases of
// a uniform array's beam, s_b its centring in samples).
// A transform of P <= 8192 points is one LDS transform; P = 16384 is
// two 8192-point halves (the inputs are zero past L <= P/2, so
// G[2k] = FFT_H(g)[k] and G[2k + 1] = FFT_H(g[n] W^n)[k], W = exp(-2 pi j / P)).
#include "kernel_common.h"

namespace fbst {

namespace {

template <typename TG, int P>
__global__ __launch_bounds__(Shape<(P > 8192 ? P / 2 : P)>::THREADS) void k_gs_spectra(
    const cx<double>* __restrict__ x, int B, int L, cx<TG>* __restrict__ G1,
    cx<TG>* __restrict__ G2, const cx<double>* __restrict__ tw, const int* __restrict__ key,
    const double* __restrict__ sb, double eps) {
  constexpr bool SPLIT = P > 8192;
  constexpr int H = SPLIT ? P / 2 : P;
  using SH = Shape<H>;
  __shared__ cx<double> lds[SH::G * SH::S];
  const int g = threadIdx.x / SH::TT, t = threadIdx.x % SH::TT;
  const int b0 = blockIdx.x * SH::G + g;
  const bool active = b0 < B;
  const int b = active ? b0 : 0;
  const cx<double>* xb = x + static_cast<size_t>(key ? key[b] : b) * L;
  const double s_b = key ? sb[b] : 0.0;
  // x_b[d], the phase computed as the host computes it
  auto xat = [&](int d) {
    const cx<double> v = xb[d];
    if (!key || d == 0) return v;
    double sn, cs;
    sincos(-2.0 * 3.141592653589793238 * eps * d / L * s_b, &sn, &cs);
    return cmul(v, cx<double>{cs, sn});
  };
  const double scale = 1.0 / (static_cast<double>(P) * sqrt(xb[0].re));
  cx<double>* buf = lds + g * SH::S;
  cx<double> v[kE];
#pragma unroll 1
  for (int which = 0; which < 2; ++which) {
    cx<TG>* dst = (which ? G2 : G1) + static_cast<size_t>(b) * P;
#pragma unroll 1
    for (int par = 0; par < (SPLIT ? 2 : 1); ++par) {
#pragma unroll
      for (int s = 0; s < kE; ++s) {
        const int i = t + s * SH::TT;
        cx<double> e{0.0, 0.0};
        if (i < L) e = which == 0 ? xat(i) : (i == 0 ? cx<double>{0.0, 0.0} : conjg(xat(L - i)));
        if constexpr (SPLIT) {
          if (par) e = cmul(e, split_twiddle<P>(tw, i));
        }
        v[s] = e;
      }
      fft<double, H, kE, -1>(v, buf, tw, t);
#pragma unroll
      for (int s = 0; s < kE; ++s) {
        const int i = t + s * SH::TT;
        const int k = SPLIT ? 2 * i + par : i;
        if (active) dst[k] = cvt<TG>(v[s] * scale);
      }
    }
  }
}

}  // namespace

template <typename TG>
hipError_t launch_gs_spectra(int P, const void* x, int B, int L, void* G1, void* G2,
                             const void* tw64, hipStream_t st, const int* key, const double* s,
                             double eps) {
  if (B < 1 || L < 1 || 2 * L > P) return hipErrorInvalidValue;
  switch (P) {
#define CASE(PP)                                                                               \
  case PP: {                                                                                   \
    using SH = Shape<(PP > 8192 ? PP / 2 : PP)>;                                               \
    hipLaunchKernelGGL((k_gs_spectra<TG, PP>), dim3((B + SH::G - 1) / SH::G),                   \
                       dim3(SH::THREADS), 0, st, (const cx<double>*)x, B, L, (cx<TG>*)G1,      \
                       (cx<TG>*)G2, (const cx<double>*)tw64, key, s, eps);                     \
    return hipGetLastError();                                                                  \
  }
    FBST_FOR_EACH_P(CASE)
#undef CASE
    default:
      break;
  }
  return hipErrorInvalidValue;
}

template hipError_t launch_gs_spectra<float>(int, const void*, int, int, void*, void*, const void*,
                                             hipStream_t, const int*, const double*, double);
template hipError_t launch_gs_spectra<double>(int, const void*, int, int, void*, void*,
                                              const void*, hipStream_t, const int*, const double*,
                                              double);

}  // namespace fbst
