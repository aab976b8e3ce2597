// Per-beam complex products on the float32 matrix cores: stage 2 in
// precomputed form and the product of beamspace nulling.
//
// Stage 2 in precomputed form (the FBST-Precompute variant, Sec. V and
// Table I): for a fixed beam set the map from w_b to the beam is the fixed
// N x L matrix K_b = F_u A_b^{-1}, so a plan may build it once and apply it
// as a matrix product.  Across the blocks of one launch that product is, per
// beam, a complex GEMM
//     beams_blk[b][n] = sum_l K_b[n][l] W[blk][b][l],
// done here on the float32 matrix cores (v_mfma_f32_16x16x4f32, float32
// operands and accumulation, so no precision is given up against the
// Gohberg-Semencul path).
//
// K is stored [L][B][N] (the output layout of the stage-2 kernel run on unit
// vectors, which is how the plan builds it): column l of K_b is contiguous in
// n.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cx.h"
#include "kernels.h"

namespace fbst {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kXCD = 8;
constexpr int PT_N = 64;    // outputs n per workgroup
#ifndef FBST_PT_B
#define FBST_PT_B 32
#endif
constexpr int PT_B = FBST_PT_B;    // blocks per workgroup (32 or 16)
constexpr int PT_KC = 32;   // basis frequencies per LDS chunk
constexpr int PT_AS = PT_N + 1;    // LDS row strides (elements): rows of consecutive lanes
constexpr int PT_BS = PT_KC + 1;   // fall in different banks

__device__ __forceinline__ int xcd_linear(int nwg) {
  const int b = blockIdx.x;
  const int x = b % kXCD, i = b / kXCD;
  const int q = nwg / kXCD, r = nwg % kXCD;
  return (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// out[blk][g][n] = sum_k K[k][g][n] in[blk][row(g)][k] for every output group
// g < NG (a beam), n < NO, k < KL.  Workgroup: one group, PT_N outputs x PT_B
// blocks, 4 waves as 2 (n) x 2 (blocks) for 32 blocks (a wave owns 32 n x 16
// blocks, two 16 x 16 tiles) or 4 (n) x 1 for 16 blocks (one tile per wave,
// twice the workgroups).  Matrix-core operand layouts (16x16x4, float32):
// A lane l holds A[l % 16][l / 16], B lane l holds B[l / 16][l % 16],
// accumulator lane l holds D[4 (l / 16) + e][l % 16], e < 4.
__global__ __launch_bounds__(256) void k_beam_product(const ProductArgs a, int n_ntiles,
                                                      int n_btiles) {
  __shared__ c32 As[PT_KC * PT_AS];   // [k][n]
  __shared__ c32 Bs[PT_B * PT_BS];    // [blk][k]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int NG = a.NG, KL = a.KL, NO = a.NO, nb = a.nb;
  // logical order: group outermost, so the workgroups sharing K_g sit on one XCD
  int w = xcd_linear(gridDim.x);
  const int bt = w % n_btiles;
  w /= n_btiles;
  const int nt = w % n_ntiles;
  const int g = w / n_ntiles;
  const int n0 = nt * PT_N, blk0 = bt * PT_B;
  const int row = a.in_map ? a.in_map[g] : (a.in_rows == 1 ? 0 : g);

  // global -> register staging of one chunk: A 64 x 32 (8 per thread),
  // B PT_B x 32 (PT_B / 8 per thread), zero outside [NO) x [KL) and [nb) x [KL)
  static_assert(PT_B == 16 || PT_B == 32, "block tile of 16 or 32");
  constexpr int BI = PT_B / 8;
  const int an = tid % PT_N, ak = tid / PT_N;          // + 4 i
  const int bk = tid % PT_KC, bb = tid / PT_KC;        // + 8 i
  const bool a_ok = n0 + an < NO;
  const c32* Kg = a.K + static_cast<size_t>(g) * NO + n0 + (a_ok ? an : 0);
  c32 ra[8], rb[BI];
  auto load_chunk = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = k0 + ak + 4 * i;
      const c32 v = Kg[static_cast<size_t>(k < KL ? k : KL - 1) * NG * NO];
      ra[i] = (a_ok && k < KL) ? v : c32{0.f, 0.f};
    }
#pragma unroll
    for (int i = 0; i < BI; ++i) {
      const int blk = blk0 + bb + 8 * i;
      const int k = k0 + bk;
      const bool ok = blk < nb && k < KL;
      const c32 v =
          a.in[(static_cast<size_t>(ok ? blk : 0) * a.in_rows + row) * KL + (ok ? k : 0)];
      rb[i] = ok ? v : c32{0.f, 0.f};
    }
    asm volatile("" ::: "memory");   // issue the chunk's loads together
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int i = 0; i < 8; ++i) As[(ak + 4 * i) * PT_AS + an] = ra[i];
#pragma unroll
    for (int i = 0; i < BI; ++i) Bs[(bb + 8 * i) * PT_BS + bk] = rb[i];
  };

  constexpr int WN = PT_B == 32 ? 2 : 4;               // waves along n
  constexpr int RT = PT_N / (16 * WN);                  // 16-row tiles per wave
  const int wn = wave % WN, wb = wave / WN;
  const int r16 = lane & 15, kq = lane >> 4;
  f32x4 accR[RT], accI[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    accR[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
    accI[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  load_chunk(0);
  for (int k0 = 0; k0 < KL; k0 += PT_KC) {
    __syncthreads();                 // the previous chunk has been consumed
    store_chunk();
    __syncthreads();
    if (k0 + PT_KC < KL) load_chunk(k0 + PT_KC);   // in flight during the products
#pragma unroll
    for (int ks = 0; ks < PT_KC / 4; ++ks) {
      const int k = 4 * ks + kq;
      const c32 bv = Bs[(16 * wb + r16) * PT_BS + k];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const c32 av = As[k * PT_AS + 16 * RT * wn + 16 * rt + r16];
        accR[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.re, bv.re, accR[rt], 0, 0, 0);
        accR[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(-av.im, bv.im, accR[rt], 0, 0, 0);
        accI[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.re, bv.im, accI[rt], 0, 0, 0);
        accI[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.im, bv.re, accI[rt], 0, 0, 0);
      }
    }
  }
  // accumulator lane l: n = n0 + 16 RT wn + 16 rt + 4 (l / 16) + e, block blk0 + 16 wb + l % 16
  const int blk = blk0 + 16 * wb + r16;
  if (blk < nb) {
    const size_t o = (static_cast<size_t>(blk) * NG + g) * NO;
    c32* dst = a.out ? a.out + o : static_cast<c32*>(a.outs.p[blk]) + static_cast<size_t>(g) * NO;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int n = n0 + 16 * RT * wn + 16 * rt + 4 * kq + e;
        if (n < NO) {
          c32 v = c32{accR[rt][e], accI[rt][e]};
          if (a.base) {
            const c32 bsv = a.base[o + n];
            v = c32{bsv.re - v.re, bsv.im - v.im};
          }
          dst[n] = v;
        }
      }
  }
}

// w[j][b][l] = (l == l0 + j), j < rows: the unit vectors whose stage-2 images
// are the columns of K.
__global__ __launch_bounds__(256) void k_unit_rows(c32* __restrict__ w, int B, int L, int l0,
                                                   int rows) {
  const size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
  const size_t total = static_cast<size_t>(rows) * B * L;
  if (i >= total) return;
  const int l = static_cast<int>(i % L);
  const int j = static_cast<int>(i / (static_cast<size_t>(B) * L));
  w[i] = c32{l == l0 + j ? 1.f : 0.f, 0.f};
}

// out[blk][q][l] = w[blk][map[q]][l]: the rows of the interferer beams.
__global__ __launch_bounds__(256) void k_gather_rows(const c32* __restrict__ w,
                                                     const int* __restrict__ map,
                                                     c32* __restrict__ out, int B, int P, int L,
                                                     int nb) {
  const size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
  const size_t total = static_cast<size_t>(nb) * P * L;
  if (i >= total) return;
  const int l = static_cast<int>(i % L);
  const size_t r = i / L;
  const int q = static_cast<int>(r % P);
  const size_t blk = r / P;
  out[i] = w[(blk * B + map[q]) * L + l];
}

// out[blk][q][l] = sum_m yhat[blk][m][l] E[q][m][l]: the beam vectors of
// arbitrary directions from stage 1a's output (the sum over sensors of
// eq. DFT_1 written out; M terms per output, float32 accumulation).
__global__ __launch_bounds__(256) void k_project_dirs(const c32* __restrict__ yhat,
                                                      const c32* __restrict__ E,
                                                      c32* __restrict__ out, int M, int P, int L,
                                                      int nb) {
  const size_t i = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x;
  const size_t total = static_cast<size_t>(nb) * P * L;
  if (i >= total) return;
  const int l = static_cast<int>(i % L);
  const size_t r = i / L;
  const int q = static_cast<int>(r % P);
  const size_t blk = r / P;
  const c32* y = yhat + blk * M * L + l;
  const c32* e = E + static_cast<size_t>(q) * M * L + l;
  float re = 0.f, im = 0.f;
  for (int m = 0; m < M; ++m) {
    const c32 a = y[static_cast<size_t>(m) * L], b = e[static_cast<size_t>(m) * L];
    re = fmaf(a.re, b.re, re);
    re = fmaf(-a.im, b.im, re);
    im = fmaf(a.re, b.im, im);
    im = fmaf(a.im, b.re, im);
  }
  out[i] = c32{re, im};
}

}  // namespace

hipError_t launch_project_dirs(const void* yhat, const void* E, void* out, int M, int P, int L,
                               int nblocks, hipStream_t st) {
  if (nblocks < 1 || M < 1 || P < 1 || L < 1 || !E) return hipErrorInvalidValue;
  const size_t total = static_cast<size_t>(nblocks) * P * L;
  const size_t grid = (total + 255) / 256;
  if (grid > 0x7fffffffULL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_project_dirs, dim3(static_cast<unsigned>(grid)), dim3(256), 0, st,
                     static_cast<const c32*>(yhat), static_cast<const c32*>(E),
                     static_cast<c32*>(out), M, P, L, nblocks);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const void* w, const int* map, void* out, int B, int P, int L,
                              int nblocks, hipStream_t st) {
  if (nblocks < 1 || B < 1 || P < 1 || L < 1 || !map) return hipErrorInvalidValue;
  const size_t total = static_cast<size_t>(nblocks) * P * L;
  const size_t grid = (total + 255) / 256;
  if (grid > 0x7fffffffULL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gather_rows, dim3(static_cast<unsigned>(grid)), dim3(256), 0, st,
                     static_cast<const c32*>(w), map, static_cast<c32*>(out), B, P, L, nblocks);
  return hipGetLastError();
}

hipError_t launch_beam_product(const ProductArgs& a, hipStream_t st) {
  if (a.nb < 1 || a.nb > MAX_LAUNCH_BLOCKS || a.NG < 1 || a.KL < 1 || a.NO < 1 || a.in_rows < 1 ||
      !a.K || !a.in)
    return hipErrorInvalidValue;
  const int n_ntiles = (a.NO + PT_N - 1) / PT_N, n_btiles = (a.nb + PT_B - 1) / PT_B;
  const long long ng = 1LL * a.NG * n_ntiles * n_btiles;
  if (ng > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_beam_product, dim3(static_cast<unsigned>(ng)), dim3(256), 0, st, a,
                     n_ntiles, n_btiles);
  return hipGetLastError();
}

hipError_t launch_precomputed_apply(const void* K, const void* w, const OutPtrs& outs, int B,
                                    int L, int N, int nblocks, hipStream_t st) {
  ProductArgs a{};
  a.K = static_cast<const c32*>(K);
  a.in = static_cast<const c32*>(w);
  a.in_rows = B;
  a.outs = outs;
  a.NG = B;
  a.KL = L;
  a.NO = N;
  a.nb = nblocks;
  return launch_beam_product(a, st);
}

hipError_t launch_unit_rows(void* w, int B, int L, int l0, int rows, hipStream_t st) {
  if (rows < 1 || B < 1 || L < 1) return hipErrorInvalidValue;
  const size_t total = static_cast<size_t>(rows) * B * L;
  const size_t grid = (total + 255) / 256;
  if (grid > 0x7fffffffULL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_unit_rows, dim3(static_cast<unsigned>(grid)), dim3(256), 0, st,
                     static_cast<c32*>(w), B, L, l0, rows);
  return hipGetLastError();
}

namespace {

// Off-grid beams by spline interpolation (Sec. VIII), tensor product over the
// beam grid (beam b = a bv + c):
//   out[blk][d][n] = sum_{i < 8, j < TV} wu[d][i] wv[d][j] beams[blk][(a0 + i) bv + c0 + j][n]
// with (a0, c0) = first[d] and (wu, wv) = w[d]; TV = 1 for a line of beams
// (bv = 1, wv = 1), 8 for a plane.
// One workgroup per 256 consecutive n of one (block, direction) row, so the
// window and its weights are uniform over the workgroup; the 8 input rows are
// read coalesced in n.  Each XCD takes a contiguous range of rows, so the
// directions that share grid beams read them through one L2.
template <typename T, int TV>
__global__ __launch_bounds__(256) void k_interp_beams(const cx<T>* __restrict__ beams,
                                                      const int* __restrict__ first,
                                                      const double* __restrict__ w,
                                                      cx<T>* __restrict__ out, int B, int bv,
                                                      int D, int N, int ntile) {
  const int wg = xcd_linear(gridDim.x);          // contiguous logical range per XCD
  const int row = wg / ntile;                    // blk * D + d
  const int n = (wg - row * ntile) * 256 + threadIdx.x;
  if (n >= N) return;
  const int d = row % D;
  const size_t blk = static_cast<size_t>(row / D);
  const int a0 = first[2 * d], c0 = first[2 * d + 1];
  const cx<T>* src = beams + (blk * B + static_cast<size_t>(a0) * bv + c0) * N + n;
  const double* wd = w + static_cast<size_t>(d) * 16;
  T re = 0, im = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
#pragma unroll
    for (int j = 0; j < TV; ++j) {
      const cx<T> a = src[(static_cast<size_t>(i) * bv + j) * N];
      const T c = static_cast<T>(wd[i] * wd[8 + j]);
      re += c * a.re;
      im += c * a.im;
    }
  }
  out[static_cast<size_t>(row) * N + n] = cx<T>{re, im};
}

// The same sum in float32 with two consecutive samples per lane (16-byte
// loads and stores; N even and both buffers 16-byte aligned).  Each sample
// takes the same operations in the same order as above, so the results are
// identical.
template <int TV>
__global__ __launch_bounds__(256) void k_interp_beams_x2(const float4* __restrict__ beams,
                                                         const int* __restrict__ first,
                                                         const double* __restrict__ w,
                                                         float4* __restrict__ out, int B, int bv,
                                                         int D, int N2, int ntile) {
  const int wg = xcd_linear(gridDim.x);
  const int row = wg / ntile;                    // blk * D + d
  const int q = (wg - row * ntile) * 256 + threadIdx.x;   // sample pair: n = 2 q, 2 q + 1
  if (q >= N2) return;
  const int d = row % D;
  const size_t blk = static_cast<size_t>(row / D);
  const int a0 = first[2 * d], c0 = first[2 * d + 1];
  const float4* src = beams + (blk * B + static_cast<size_t>(a0) * bv + c0) * N2 + q;
  const double* wd = w + static_cast<size_t>(d) * 16;
  float r0 = 0, i0 = 0, r1 = 0, i1 = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
#pragma unroll
    for (int j = 0; j < TV; ++j) {
      const float4 a = src[(static_cast<size_t>(i) * bv + j) * N2];
      const float c = static_cast<float>(wd[i] * wd[8 + j]);
      r0 += c * a.x;
      i0 += c * a.y;
      r1 += c * a.z;
      i1 += c * a.w;
    }
  }
  out[static_cast<size_t>(row) * N2 + q] = make_float4(r0, i0, r1, i1);
}

// Beamspace vectors at directions, spline-interpolated from the grid's
// (Sec. VIII, the paper's off-grid form), with the reference point moved to
// the array's centre c for the interpolation:
//   out[blk][d][l] = sum_{i < 8, j < TV} wu[i] wv[j]
//                    exp(j (theta_x[l] (fu - i) + theta_y[l] (fv - j)))
//                    W[blk][(a0 + i) bv + c0 + j][l]
// where theta_x[l] = a_l c_x du (u - u_{a0+i} = (fu - i) du) and likewise
// along v; (a0, c0) = first[d], (fu, fv) = frac[d].  The per-tap phases are
// formed in float64 and reduced to [-pi, pi] before the float32 sine and
// cosine.  One workgroup per 256 consecutive l of one (block, direction)
// row, XCD-contiguous like k_interp_beams.
template <int TV>
__global__ __launch_bounds__(256) void k_interp_vectors(const c32* __restrict__ W,
                                                        const int* __restrict__ first,
                                                        const double* __restrict__ w,
                                                        const double* __restrict__ frac,
                                                        const double* __restrict__ theta,
                                                        c32* __restrict__ out, int B, int bv,
                                                        int D, int L, int ntile) {
  const int wg = xcd_linear(gridDim.x);
  const int row = wg / ntile;                    // blk * D + d
  const int l = (wg - row * ntile) * 256 + threadIdx.x;
  if (l >= L) return;
  const int d = row % D;
  const size_t blk = static_cast<size_t>(row / D);
  const int a0 = first[2 * d], c0 = first[2 * d + 1];
  const double* wd = w + static_cast<size_t>(d) * 16;
  const double twopi = 6.283185307179586476925;
  auto rot = [&](double ph) {
    ph -= twopi * rint(ph * (1.0 / twopi));
    float sn, cs;
    sincosf(static_cast<float>(ph), &sn, &cs);
    return c32{cs, sn};
  };
  c32 rx[8], ry[TV];
  const double fu = frac[2 * d], tx = theta[l];
#pragma unroll
  for (int i = 0; i < 8; ++i) rx[i] = rot(tx * (fu - i));
  if (TV > 1) {
    const double fv = frac[2 * d + 1], ty = theta[L + l];
#pragma unroll
    for (int j = 0; j < TV; ++j) ry[j] = rot(ty * (fv - j));
  } else {
    ry[0] = c32{1.0f, 0.0f};
  }
  const c32* src = W + (blk * B + static_cast<size_t>(a0) * bv + c0) * L + l;
  float re = 0, im = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
#pragma unroll
    for (int j = 0; j < TV; ++j) {
      const c32 a = src[(static_cast<size_t>(i) * bv + j) * L];
      const c32 r = (TV > 1) ? c32{rx[i].re * ry[j].re - rx[i].im * ry[j].im,
                                   rx[i].re * ry[j].im + rx[i].im * ry[j].re}
                             : rx[i];
      const float c = static_cast<float>(wd[i] * wd[8 + j]);
      re += c * (r.re * a.re - r.im * a.im);
      im += c * (r.re * a.im + r.im * a.re);
    }
  }
  out[static_cast<size_t>(row) * L + l] = c32{re, im};
}

}  // namespace

hipError_t launch_interp_beams(const void* beams, const int* first, const double* w, void* out,
                               int B, int bv, int D, int N, int nblocks, bool fp64,
                               hipStream_t st) {
  if (nblocks < 1 || bv < 1 || B % bv != 0 || B / bv < 8 || (bv > 1 && bv < 8) || D < 1 || N < 1)
    return hipErrorInvalidValue;
  const long long ntile = (N + 255) / 256;
  const long long grid = 1LL * nblocks * D * ntile;
  if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 g(static_cast<unsigned>(grid)), b(256);
  const int nt = static_cast<int>(ntile);
  if (fp64) {
    auto in = static_cast<const cx<double>*>(beams);
    auto o = static_cast<cx<double>*>(out);
    if (bv > 1) hipLaunchKernelGGL((k_interp_beams<double, 8>), g, b, 0, st, in, first, w, o, B, bv, D, N, nt);
    else hipLaunchKernelGGL((k_interp_beams<double, 1>), g, b, 0, st, in, first, w, o, B, bv, D, N, nt);
  } else if (N % 2 == 0 && reinterpret_cast<uintptr_t>(beams) % 16 == 0 &&
             reinterpret_cast<uintptr_t>(out) % 16 == 0) {
    const int n2 = N / 2;
    const long long nt2 = (n2 + 255) / 256;
    const dim3 g2(static_cast<unsigned>(1LL * nblocks * D * nt2));
    auto in = static_cast<const float4*>(beams);
    auto o = static_cast<float4*>(out);
    if (bv > 1)
      hipLaunchKernelGGL((k_interp_beams_x2<8>), g2, b, 0, st, in, first, w, o, B, bv, D, n2,
                         static_cast<int>(nt2));
    else
      hipLaunchKernelGGL((k_interp_beams_x2<1>), g2, b, 0, st, in, first, w, o, B, bv, D, n2,
                         static_cast<int>(nt2));
  } else {
    auto in = static_cast<const cx<float>*>(beams);
    auto o = static_cast<cx<float>*>(out);
    if (bv > 1) hipLaunchKernelGGL((k_interp_beams<float, 8>), g, b, 0, st, in, first, w, o, B, bv, D, N, nt);
    else hipLaunchKernelGGL((k_interp_beams<float, 1>), g, b, 0, st, in, first, w, o, B, bv, D, N, nt);
  }
  return hipGetLastError();
}

hipError_t launch_interp_vectors(const void* W, const int* first, const double* w,
                                 const double* frac, const double* theta, void* out, int B,
                                 int bv, int D, int L, int nblocks, hipStream_t st) {
  if (nblocks < 1 || bv < 1 || B % bv != 0 || B / bv < 8 || (bv > 1 && bv < 8) || D < 1 || L < 1)
    return hipErrorInvalidValue;
  const long long ntile = (L + 255) / 256;
  const long long grid = 1LL * nblocks * D * ntile;
  if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 g(static_cast<unsigned>(grid)), b(256);
  auto in = static_cast<const c32*>(W);
  auto o = static_cast<c32*>(out);
  if (bv > 1)
    hipLaunchKernelGGL((k_interp_vectors<8>), g, b, 0, st, in, first, w, frac, theta, o, B, bv, D,
                       L, static_cast<int>(ntile));
  else
    hipLaunchKernelGGL((k_interp_vectors<1>), g, b, 0, st, in, first, w, frac, theta, o, B, bv, D,
                       L, static_cast<int>(ntile));
  return hipGetLastError();
}

}  // namespace fbst
