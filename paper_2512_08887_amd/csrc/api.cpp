// C ABI of libfbst.so (declared in include/fbst.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <string>
#include <vector>

#include "fft_lds.h"
#include "kernels.h"
#include "plan.h"

namespace {

thread_local std::string g_last_error;

fbst_status fail(fbst_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

}  // namespace

void fbst::set_last_error(const std::string& msg) { g_last_error = msg; }

namespace {

fbst_status hip_fail(hipError_t e, const char* what) {
  return fail(FBST_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool stage1_double(const fbst::Params& p) { return p.prec == FBST_PREC_FP64; }
bool stage2_double(const fbst::Params& p) {
  return p.prec == FBST_PREC_FP64 || p.prec == FBST_PREC_FP64_STAGE2;
}
size_t s1_elem(const fbst::Params& p) { return stage1_double(p) ? 16 : 8; }
bool fp32_stage2(const fbst::Params& p) {
  return p.prec == FBST_PREC_FP32 || p.prec == FBST_PREC_BF16_SPLIT ||
         p.prec == FBST_PREC_FP16_SPLIT;
}
size_t s2_elem(const fbst::Params& p) { return stage2_double(p) ? 16 : 8; }
// float64 stage 2 whose transforms exceed the LDS: each split into two halves
bool split_stage2(const fbst::Params& p) { return stage2_double(p) && p.p3 > 8192; }

// Elements per block of stage 1b's scratch z: a grid's x-axis output
// [bu][my][L]; for arbitrary positions the oversampled grid [nfx][nfy][L]
// and, in 2-D, the x-axis output [bu][nfy][L].
size_t z_elems(const fbst::Params& p) {
  if (p.kind == FBST_GRID) return static_cast<size_t>(p.bu) * p.my * p.L;
  if (p.kind == FBST_ARBITRARY) {
    const size_t nfy = p.p2y ? p.p2y : 1;
    return (static_cast<size_t>(p.p2x) * nfy + (p.p2y ? static_cast<size_t>(p.bu) * nfy : 0)) * p.L;
  }
  return 0;
}

// Elements per block of the refined stage 2's first solution beta_1 [B][L]
// (float32 stage 2 only, so the stage-1 element size is the stage-2 one).
size_t refine_elems(const fbst::Params& p) {
  return (p.flags & FBST_FLAG_STAGE2_REFINE) ? static_cast<size_t>(p.B) * p.L : 0;
}

// Workspace of one block: [yhat M L | w B L | z | beta_1] in the stage-1 type.
size_t ws_per_block(const fbst::Params& p) {
  const size_t elems = (static_cast<size_t>(p.M) + p.B) * p.L + z_elems(p) + refine_elems(p);
  return elems * s1_elem(p);
}

size_t align_up(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Staging of host tables into one device allocation.
struct Upload {
  std::vector<unsigned char> blob;
  size_t add_ints(const std::vector<int>& v) {
    const size_t off = align_up(blob.size());
    blob.resize(off + v.size() * sizeof(int));
    if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(int));
    return off;
  }
  size_t add_doubles(const std::vector<double>& v) {
    const size_t off = align_up(blob.size());
    blob.resize(off + v.size() * sizeof(double));
    if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(double));
    return off;
  }
  size_t add(const std::vector<fbst::zd>& v, bool as_double) {
    const size_t off = align_up(blob.size());
    const size_t bytes = v.size() * (as_double ? 16 : 8);
    blob.resize(off + bytes);
    if (as_double) {
      std::memcpy(blob.data() + off, v.data(), bytes);
    } else {
      float* f = reinterpret_cast<float*>(blob.data() + off);
      for (size_t i = 0; i < v.size(); ++i) {
        f[2 * i] = static_cast<float>(v[i].real());
        f[2 * i + 1] = static_cast<float>(v[i].imag());
      }
    }
    return off;
  }
};

// Per-pass twiddle tables of every transform size (layout in fft_lds.h):
// entry tw_offset(P, NS) + (r - 1) NS + k = exp(-2 pi j r k / (NS R)); for
// the radix-16 passes after the first, entry TW_MERGED + tw_offset(P, NS) +
// i NS + k holds the i-th merged factor f of k as (Re f, Im f / Re f).
std::vector<fbst::zd> twiddles() {
  std::vector<fbst::zd> tw(fbst::TW_TABLE, fbst::zd(0.0, 0.0));
  const double pi = 3.141592653589793238462643383279502884;
  // exp(-2 pi j m / D) as (c, t), |c| held at least 2^-40
  auto merged = [&](long long m, long long D) {
    const double a = 2.0 * pi * static_cast<double>(((m % D) + D) % D) / static_cast<double>(D);
    double c = std::cos(a);
    const double s = -std::sin(a);
    const double cmin = std::ldexp(1.0, -40);
    if (std::fabs(c) < cmin) c = std::signbit(c) ? -cmin : cmin;
    return fbst::zd(c, s / c);
  };
  for (int P = 32; P <= fbst::PMAX; P *= 2) {
    for (int NS = 1; NS < P;) {
      const int R = std::min(fbst::FFT_E, P / NS);
      if (NS > 1) {
        const int off = fbst::tw_offset(P, NS);
        const long long NR = 1LL * NS * R;
        for (int r = 1; r < R; ++r)
          for (int k = 0; k < NS; ++k) {
            const double a = 2.0 * pi * static_cast<double>((1LL * r * k) % NR) / static_cast<double>(NR);
            tw[off + (r - 1) * NS + k] = fbst::zd(std::cos(a), -std::sin(a));
          }
        if (R == 16) {
          // angles in units of 2 pi / (16 NS): psi = w^{4k}, om = w^k w_16^{k1},
          // i^-1 = 4 NS units
          const long long D = 16LL * NS, q = 4LL * NS;
          fbst::zd* m = tw.data() + fbst::TW_MERGED + off;
          for (int k = 0; k < NS; ++k) {
            m[0 * NS + k] = merged(8LL * k, D);
            m[1 * NS + k] = merged(4LL * k, D);
            m[2 * NS + k] = merged(4LL * k + q, D);
            for (int k1 = 0; k1 < 4; ++k1) {
              const long long o = k + 1LL * NS * k1;
              m[(3 + 3 * k1) * NS + k] = merged(2 * o, D);
              m[(4 + 3 * k1) * NS + k] = merged(o, D);
              m[(5 + 3 * k1) * NS + k] = merged(o + q, D);
            }
          }
        }
      }
      NS *= R;
    }
  }
  return tw;
}

fbst_status upload(fbst_plan* pl) {
  const fbst::Params& p = pl->p;
  const bool d1 = stage1_double(p), d2 = stage2_double(p);
  fbst::HostTables& h = pl->host;
  Upload up;
  const std::vector<fbst::zd> tw = twiddles();
  const size_t o_tw1 = up.add(tw, d1);
  const size_t o_tw2 = (d1 == d2) ? o_tw1 : up.add(tw, d2);
  const size_t o_pre1 = up.add(h.pre1, d1), o_H1 = up.add(h.H1, d1), o_post1 = up.add(h.post1, d1);
  const size_t o_H1a = up.add(h.H1a, d1), o_H1b = up.add(h.H1b, d1);
  const size_t o_axp = up.add(h.ax.pre, d1), o_axH = up.add(h.ax.H, d1), o_axq = up.add(h.ax.post, d1);
  size_t o_ayp = 0, o_ayH = 0, o_ayq = 0;
  if (p.kind == FBST_GRID) {
    o_ayp = up.add(h.ay.pre, d1);
    o_ayH = up.add(h.ay.H, d1);
    o_ayq = up.add(h.ay.post, d1);
  }
  const size_t o_nup = up.add(h.nu_pre, d1), o_nux = up.add(h.nu_posx, d1),
               o_nuy = up.add(h.nu_posy, d1), o_nucx = up.add(h.nu_cx, d1),
               o_nucy = up.add(h.nu_cy, d1), o_nuo = up.add_ints(h.nu_order);
  const size_t o_G1 = up.add(h.G1, d2), o_G2 = up.add(h.G2, d2);
  const size_t o_pre3 = up.add(h.pre3, d2), o_H3 = up.add(h.H3, d2), o_post3 = up.add(h.post3, d2);
  const size_t o_CA = up.add(h.CA, d2);
  const size_t tables = align_up(up.blob.size());
  const size_t total = tables + align_up(pl->ws_bytes_per_block) + pl->ws_fixed_bytes;

  hipError_t e = hipGetDevice(&pl->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  void* dev = nullptr;
  e = hipMalloc(&dev, total);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(FBST_E_NOMEM, "hipMalloc of " + std::to_string(total) + " bytes of plan tables failed");
  }
  e = hipMemcpy(dev, up.blob.data(), up.blob.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(dev);
    return hip_fail(e, "hipMemcpy of plan tables");
  }
  unsigned char* b = static_cast<unsigned char*>(dev);
  pl->dev = dev;
  pl->dev_bytes = total;
  pl->tw1 = b + o_tw1;
  pl->tw2 = b + o_tw2;
  pl->pre1 = b + o_pre1;
  pl->H1 = b + o_H1;
  pl->post1 = b + o_post1;
  if (p.p1s) {
    pl->H1a = b + o_H1a;
    pl->H1b = b + o_H1b;
  }
  pl->axp = b + o_axp;
  pl->axH = b + o_axH;
  pl->axq = b + o_axq;
  if (p.kind == FBST_GRID) {
    pl->ayp = b + o_ayp;
    pl->ayH = b + o_ayH;
    pl->ayq = b + o_ayq;
  }
  if (p.kind == FBST_ARBITRARY) {
    pl->nu_pre = b + o_nup;
    pl->nu_posx = b + o_nux;
    pl->nu_cx = b + o_nucx;
    pl->nu_order = reinterpret_cast<const int*>(b + o_nuo);
    if (p.p2y) {
      pl->nu_posy = b + o_nuy;
      pl->nu_cy = b + o_nucy;
    }
  }
  pl->G1 = b + o_G1;
  pl->G2 = b + o_G2;
  pl->pre3 = b + o_pre3;
  pl->H3 = b + o_H3;
  pl->post3 = b + o_post3;
  if (p.flags & FBST_FLAG_STAGE2_REFINE) pl->CA = b + o_CA;
  pl->own_ws = b + tables;
  return FBST_OK;
}

size_t io_elem(const fbst::Params& p) { return p.prec == FBST_PREC_FP64 ? 16 : 8; }

template <typename T1>
hipError_t run_stage0(const fbst_plan* pl, int nb, const fbst::InPtrs& xs, void* yhat,
                      hipStream_t st) {
  const fbst::Params& p = pl->p;
  if (p.prec == FBST_PREC_BF16_SPLIT || p.prec == FBST_PREC_FP16_SPLIT)
    return fbst::launch_time_czt_mfma(p.p1, p.prec == FBST_PREC_FP16_SPLIT, xs, nb, yhat, pl->pre1,
                                      pl->H1, pl->post1, pl->tw1, p.M, p.N, p.L, st);
  if (p.p1s)
    return fbst::launch_time_czt_split<T1>(p.p1s, xs, nb, yhat, pl->pre1, pl->H1a, pl->H1b,
                                           pl->post1, pl->tw1, p.M, p.N, p.L, p.ls1, st);
  return fbst::launch_time_czt<T1>(p.p1, xs, nb, yhat, pl->pre1, pl->H1, pl->post1, pl->tw1, p.M,
                                   p.N, p.L, st);
}

template <typename T1>
hipError_t run_stage1(const fbst_plan* pl, int nb, const void* yhat, void* w, void* z,
                      hipStream_t st) {
  const fbst::Params& p = pl->p;
  const int tile = (pl->k3_variant.load(std::memory_order_relaxed) >> 4) & 3;
  if (p.kind == FBST_LINE) {
    return fbst::launch_axis_czt<T1>(p.p2x, yhat, w, pl->axp, pl->axH, pl->axq, pl->tw1, p.M, p.B,
                                     1, 1, p.L, nb, st, tile);
  }
  if (p.kind == FBST_ARBITRARY) {
    // spread yhat onto the oversampled grid z [nb][nfx][nfy][L]; 1-D: the x
    // axis straight to w; 2-D: x axis to z2 [nb][1][bu][nfy][L], then the y
    // axis on [nb][bu][nfy][1][L] -> w [nb][bu][bv][1][L]
    const int nfy = p.p2y ? p.p2y : 1;
    if (!p.p2y && p.p2x >= 256 && p.p2x <= 4096 && !(p.flags & FBST_FLAG_NU_UNFUSED))
      return fbst::launch_nu_line_fused<T1>(p.nuw, p.p2x, yhat, w, pl->nu_pre, pl->nu_posx,
                                            pl->nu_order, pl->nu_lanes, pl->nu_cx, pl->tw1, p.M,
                                            p.bu, p.nu_beta, p.L, nb, st);
    if (p.p2x == 32 && p.p2y == 32 && !(p.flags & FBST_FLAG_NU_UNFUSED))
      return fbst::launch_nu_plane_fused<T1>(p.nuw, p.p2x, p.p2y, yhat, w, pl->nu_pre, pl->nu_posx,
                                             pl->nu_posy, pl->nu_cx, pl->nu_cy, pl->tw1, p.M, p.bu,
                                             p.bv, p.nu_beta, p.L, nb, st);
    hipError_t e = fbst::launch_nu_spread<T1>(p.nuw, yhat, z, pl->nu_pre, pl->nu_posx, pl->nu_posy,
                                              pl->nu_order, pl->nu_lanes, p.M, p.p2x, nfy,
                                              p.nu_beta, p.L, nb, st);
    if (e != hipSuccess) return e;
    if (!p.p2y)
      return fbst::launch_axis_dft<T1>(p.p2x, z, w, pl->nu_cx, pl->tw1, p.bu, 1, 1, p.L, nb, st);
    void* z2 = static_cast<unsigned char*>(z) +
               static_cast<size_t>(nb) * p.p2x * nfy * p.L * sizeof(T1) * 2;
    e = fbst::launch_axis_dft<T1>(p.p2x, z, z2, pl->nu_cx, pl->tw1, p.bu, 1, nfy, p.L, nb, st);
    if (e != hipSuccess) return e;
    return fbst::launch_axis_dft<T1>(nfy, z2, w, pl->nu_cy, pl->tw1, p.bv, p.bu, 1, p.L, nb, st);
  }
  // grid: x axis on [nb][1][mx][my][L] -> z [nb][1][bu][my][L], then the
  // y axis on [nb][bu][my][1][L] -> w [nb][bu][bv][1][L]
  hipError_t e = fbst::launch_axis_czt<T1>(p.p2x, yhat, z, pl->axp, pl->axH, pl->axq, pl->tw1,
                                           p.mx, p.bu, 1, p.my, p.L, nb, st, tile);
  if (e != hipSuccess) return e;
  return fbst::launch_axis_czt<T1>(p.p2y, z, w, pl->ayp, pl->ayH, pl->ayq, pl->tw1, p.my, p.bv,
                                   p.bu, 1, p.L, nb, st, tile);
}

// bt: room for beta_1 of nb blocks ([nb][B][L] complex64) when the plan
// refines its stage 2; the split float64 stage 2's scratch (ws_fixed_bytes)
// when its transforms exceed the LDS; else unused.
hipError_t run_stage2(const fbst_plan* pl, int nb, const void* w, const fbst::OutPtrs& outs,
                      void* bt, hipStream_t st) {
  const fbst::Params& p = pl->p;
  if (pl->K) return fbst::launch_precomputed_apply(pl->K, w, outs, p.B, p.L, p.N, nb, st);
  if (split_stage2(p)) {
    if (p.prec == FBST_PREC_FP64)
      return fbst::launch_toeplitz_fu_split<double, double, double>(
          p.p3, w, outs, pl->G1, pl->G2, pl->pre3, pl->H3, pl->post3, pl->tw2, bt, p.B, p.L, p.N,
          nb, st);
    return fbst::launch_toeplitz_fu_split<double, float, float>(
        p.p3, w, outs, pl->G1, pl->G2, pl->pre3, pl->H3, pl->post3, pl->tw2, bt, p.B, p.L, p.N,
        nb, st);
  }
  const int var = pl->k3_variant.load(std::memory_order_relaxed) & 15;
  if (pl->CA)
    return fbst::launch_toeplitz_fu_refined(p.p3, w, outs, pl->G1, pl->G2, pl->pre3, pl->H3,
                                            pl->post3, pl->tw2, pl->CA, bt, p.B, p.L, p.N, nb, st);
  switch (p.prec) {
    case FBST_PREC_FP64:
      return fbst::launch_toeplitz_fu<double, double, double>(p.p3, w, outs, pl->G1, pl->G2,
                                                              pl->pre3, pl->H3, pl->post3, pl->tw2,
                                                              p.B, p.L, p.N, nb, st);
    case FBST_PREC_FP64_STAGE2:
      return fbst::launch_toeplitz_fu<double, float, float>(p.p3, w, outs, pl->G1, pl->G2,
                                                            pl->pre3, pl->H3, pl->post3, pl->tw2,
                                                            p.B, p.L, p.N, nb, st);
    default:
      return fbst::launch_toeplitz_fu<float, float, float>(p.p3, w, outs, pl->G1, pl->G2,
                                                           pl->pre3, pl->H3, pl->post3, pl->tw2,
                                                           p.B, p.L, p.N, nb, st, var);
  }
}

// Stage 2 in precomputed form: K_b = F_u A_b^{-1} for every beam, built on
// the device by the Gohberg-Semencul kernel applied to the unit vectors e_l
// (block j of a launch carries e_{l0 + j} for every beam, and its output
// block is column l0 + j of every K_b).  The build runs in float64
// arithmetic whatever the plan's stage-2 precision (float64 copies of the
// stage-2 tables are staged for it when the plan's are float32): it is a
// one-time cost, and the product then adds only float32 rounding, so the
// precomputed stage 2 is at least as accurate as the plan's own.
fbst_status build_precomputed(fbst_plan* pl) {
  const fbst::Params& p = pl->p;
  const size_t kbytes = static_cast<size_t>(p.L) * p.B * p.N * 8;
  const int chunk = 64;    // unit-vector blocks per launch (bounds the staging buffer)
  const void *tw = pl->tw2, *g1 = pl->G1, *g2 = pl->G2, *pre = pl->pre3, *h3 = pl->H3,
             *post = pl->post3;
  void* d64 = nullptr;
  if (!stage2_double(p)) {
    const fbst::HostTables& h = pl->host;
    Upload up;
    const size_t o_tw = up.add(twiddles(), true), o_g1 = up.add(h.G1, true),
                 o_g2 = up.add(h.G2, true), o_pre = up.add(h.pre3, true),
                 o_h3 = up.add(h.H3, true), o_post = up.add(h.post3, true);
    hipError_t e = hipMalloc(&d64, up.blob.size());
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(FBST_E_NOMEM, "hipMalloc of the float64 stage-2 tables failed");
    }
    e = hipMemcpy(d64, up.blob.data(), up.blob.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(d64);
      return hip_fail(e, "hipMemcpy of the float64 stage-2 tables");
    }
    const unsigned char* b = static_cast<const unsigned char*>(d64);
    tw = b + o_tw;
    g1 = b + o_g1;
    g2 = b + o_g2;
    pre = b + o_pre;
    h3 = b + o_h3;
    post = b + o_post;
  }
  void* K = nullptr;
  void* unit = nullptr;
  hipError_t e = hipMalloc(&K, kbytes);
  if (e == hipSuccess) e = hipMalloc(&unit, static_cast<size_t>(chunk) * p.B * p.L * 8);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (K) (void)hipFree(K);
    if (d64) (void)hipFree(d64);
    return fail(FBST_E_NOMEM, "hipMalloc of " + std::to_string(kbytes) + " bytes of K failed");
  }
  const hipStream_t st = nullptr;
  for (int l0 = 0; l0 < p.L && e == hipSuccess; l0 += chunk) {
    const int n = (p.L - l0 < chunk) ? p.L - l0 : chunk;
    fbst::OutPtrs outs{};
    for (int j = 0; j < n; ++j)
      outs.p[j] = static_cast<unsigned char*>(K) + static_cast<size_t>(l0 + j) * p.B * p.N * 8;
    e = fbst::launch_unit_rows(unit, p.B, p.L, l0, n, st);
    if (e == hipSuccess)
      e = fbst::launch_toeplitz_fu<double, float, float>(p.p3, unit, outs, g1, g2, pre, h3, post,
                                                         tw, p.B, p.L, p.N, n, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(unit);
  if (d64) (void)hipFree(d64);
  if (e != hipSuccess) {
    (void)hipFree(K);
    return hip_fail(e, "building the precomputed stage 2");
  }
  pl->K = K;
  pl->K_bytes = kbytes;
  pl->dev_bytes += kbytes;
  return FBST_OK;
}

}  // namespace

namespace fbst {

// Whole path for nb <= MAX_LAUNCH_BLOCKS blocks with inputs xs, outputs outs
// and the workspace [yhat | w | z] of nb blocks.
hipError_t run_blocks(const fbst_plan* pl, int nb, const InPtrs& xs, const OutPtrs& outs, void* ws,
                      hipStream_t st) {
  const Params& p = pl->p;
  const size_t e1 = s1_elem(p);
  unsigned char* base = static_cast<unsigned char*>(ws);
  void* yhat = base;
  void* w = base + static_cast<size_t>(nb) * p.M * p.L * e1;
  void* z = static_cast<unsigned char*>(w) + static_cast<size_t>(nb) * p.B * p.L * e1;
  const bool d1 = stage1_double(p);
  hipError_t e = d1 ? run_stage0<double>(pl, nb, xs, yhat, st) : run_stage0<float>(pl, nb, xs, yhat, st);
  if (e != hipSuccess) return e;
  e = d1 ? run_stage1<double>(pl, nb, yhat, w, z, st) : run_stage1<float>(pl, nb, yhat, w, z, st);
  if (e != hipSuccess) return e;
  // beta_1 (inside the per-block part), or the split stage 2's scratch right
  // after the nb blocks' part (ws_fixed_bytes; refine_elems is then 0)
  void* bt = static_cast<unsigned char*>(z) + static_cast<size_t>(nb) * z_elems(p) * e1;
  return run_stage2(pl, nb, w, outs, bt, st);
}

// Whole path for nb contiguous blocks, at most `chunk` (<= MAX_LAUNCH_BLOCKS) per launch.
hipError_t run_contiguous(const fbst_plan* pl, int nb, int chunk, const void* x, void* beams,
                          void* ws, hipStream_t st) {
  const Params& p = pl->p;
  const size_t in_blk = static_cast<size_t>(p.M) * p.N * io_elem(p);
  const size_t out_blk = static_cast<size_t>(p.B) * p.N * io_elem(p);
  for (int b0 = 0; b0 < nb; b0 += chunk) {
    const int n = (nb - b0 < chunk) ? nb - b0 : chunk;
    InPtrs xs{};
    OutPtrs outs{};
    for (int i = 0; i < n; ++i) {
      xs.p[i] = static_cast<const unsigned char*>(x) + (b0 + i) * in_blk;
      outs.p[i] = static_cast<unsigned char*>(beams) + (b0 + i) * out_blk;
    }
    hipError_t e = run_blocks(pl, n, xs, outs, ws, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace fbst

namespace {

// Workspace of one nulled block: the path's own, then the interferers' rows
// of W and the nulled W, [P][L] and [B][L] complex64.
size_t nulled_ws_per_block(const fbst_plan* pl, const fbst_nulls* nl) {
  const fbst::Params& p = pl->p;
  return align_up(pl->ws_bytes_per_block) + static_cast<size_t>(nl->P + p.B) * p.L * 8;
}

// Whole path of nb blocks with the interferers nulled in beamspace
// (eq. interfer_beam_space): after stage 1, the interferers' beam vectors w_q
// are gathered from W (on-grid) or projected from Yhat (any direction),
// w~_b = w_b - sum_q G_{b,q} w_q (one product over the P L stacked rows), and
// stage 2 runs on w~.
hipError_t run_blocks_nulled(const fbst_plan* pl, const fbst_nulls* nl, int nb,
                             const fbst::InPtrs& xs, const fbst::OutPtrs& outs, void* ws,
                             hipStream_t st) {
  const fbst::Params& p = pl->p;
  unsigned char* base = static_cast<unsigned char*>(ws);
  void* yhat = base;
  void* w = base + static_cast<size_t>(nb) * p.M * p.L * 8;
  void* z = static_cast<unsigned char*>(w) + static_cast<size_t>(nb) * p.B * p.L * 8;
  auto* wq = reinterpret_cast<fbst::c32*>(base + align_up(pl->ws_bytes_per_block * nb));
  fbst::c32* wt = wq + static_cast<size_t>(nb) * nl->P * p.L;
  hipError_t e = run_stage0<float>(pl, nb, xs, yhat, st);
  if (e == hipSuccess) e = run_stage1<float>(pl, nb, yhat, w, z, st);
  if (e == hipSuccess) {
    if (nl->map)
      e = fbst::launch_gather_rows(w, nl->map, wq, p.B, nl->P, p.L, nb, st);
    else if (nl->E)
      e = fbst::launch_project_dirs(yhat, nl->E, wq, p.M, nl->P, p.L, nb, st);
    else
      e = fbst::launch_interp_vectors(w, nl->vi.first, nl->vi.w, nl->vi.frac, nl->vi.theta, wq,
                                      p.B, p.bv, nl->P, p.L, nb, st);
  }
  if (e != hipSuccess) return e;
  fbst::ProductArgs c{};
  c.K = static_cast<const fbst::c32*>(nl->G);
  c.in = wq;
  c.in_rows = 1;
  c.out = wt;
  c.base = static_cast<const fbst::c32*>(w);
  c.NG = p.B;
  c.KL = nl->P * p.L;
  c.NO = p.L;
  c.nb = nb;
  e = fbst::launch_beam_product(c, st);
  if (e != hipSuccess) return e;
  void* bt = pl->ws_fixed_bytes ? base + static_cast<size_t>(nb) * nulled_ws_per_block(pl, nl)
                                : static_cast<unsigned char*>(z) + static_cast<size_t>(nb) * z_elems(p) * 8;
  return run_stage2(pl, nb, wt, outs, bt, st);
}

fbst_status check_exec(const fbst_plan* plan) {
  if (!plan) return fail(FBST_E_INVALID, "plan is NULL");
  if (plan->host_only) return fail(FBST_E_INVALID, "plan was created host-only");
  return FBST_OK;
}

// Beams at the directions of dr for nb blocks: stage 1a, the projection of
// each direction's beam vector from Yhat, and b_d = K_d w_d on the matrix
// cores (outputs [nb][D][N] at out).
hipError_t run_blocks_directions(const fbst_plan* pl, const fbst_directions* dr, int nb,
                                 const fbst::InPtrs& xs, void* out, void* ws, hipStream_t st) {
  const fbst::Params& p = pl->p;
  unsigned char* base = static_cast<unsigned char*>(ws);
  void* yhat = base;
  hipError_t e = run_stage0<float>(pl, nb, xs, yhat, st);
  fbst::c32* wd = nullptr;
  if (dr->E) {                                 // w_d projected from Yhat
    wd = reinterpret_cast<fbst::c32*>(base + align_up(static_cast<size_t>(nb) * p.M * p.L * 8));
    if (e == hipSuccess) e = fbst::launch_project_dirs(yhat, dr->E, wd, p.M, dr->D, p.L, nb, st);
  } else {                                     // w_d interpolated from the grid's W
    void* w = base + static_cast<size_t>(nb) * p.M * p.L * 8;
    void* z = static_cast<unsigned char*>(w) + static_cast<size_t>(nb) * p.B * p.L * 8;
    wd = reinterpret_cast<fbst::c32*>(base + align_up(pl->ws_bytes_per_block * nb));
    if (e == hipSuccess) e = run_stage1<float>(pl, nb, yhat, w, z, st);
    if (e == hipSuccess)
      e = fbst::launch_interp_vectors(w, dr->vi.first, dr->vi.w, dr->vi.frac, dr->vi.theta, wd,
                                      p.B, p.bv, dr->D, p.L, nb, st);
  }
  if (e != hipSuccess) return e;
  fbst::ProductArgs a{};
  a.K = static_cast<const fbst::c32*>(dr->K);
  a.in = wd;
  a.in_rows = dr->D;
  a.out = static_cast<fbst::c32*>(out);
  a.NG = dr->D;
  a.KL = p.L;
  a.NO = p.N;
  a.nb = nb;
  return fbst::launch_beam_product(a, st);
}

size_t directions_ws_per_block(const fbst_plan* pl, const fbst_directions* dr) {
  const fbst::Params& p = pl->p;
  const size_t front = dr->E ? static_cast<size_t>(p.M) * p.L * 8 : pl->ws_bytes_per_block;
  return align_up(front) + static_cast<size_t>(dr->D) * p.L * 8;
}

// Interpolation table of beamspace vectors at directions (ud, vd) added to
// an upload; offsets returned for set_vector_interp.
struct VIOffsets {
  size_t first = 0, w = 0, frac = 0, theta = 0;
};

fbst_status add_vector_interp(const fbst_plan* plan, const std::vector<double>& ud,
                              const std::vector<double>& vd, Upload* up, VIOffsets* o) {
  std::vector<int> first;
  std::vector<double> w, frac, theta;
  std::string msg;
  const fbst_status s = fbst::build_interp_table(plan->p, ud, vd, &first, &w, &msg, &frac);
  if (s != FBST_OK) return fail(s, msg);
  fbst::reference_phase_rates(plan->p, &theta);
  o->first = up->add_ints(first);
  o->w = up->add_doubles(w);
  o->frac = up->add_doubles(frac);
  o->theta = up->add_doubles(theta);
  return FBST_OK;
}

VectorInterp vector_interp_at(const void* dev, const VIOffsets& o) {
  const unsigned char* b = static_cast<const unsigned char*>(dev);
  VectorInterp vi;
  vi.first = reinterpret_cast<const int*>(b + o.first);
  vi.w = reinterpret_cast<const double*>(b + o.w);
  vi.frac = reinterpret_cast<const double*>(b + o.frac);
  vi.theta = reinterpret_cast<const double*>(b + o.theta);
  return vi;
}

// Nulling tables for n on-grid interferers (beam indices qs) or for n
// explicit directions (u, v; qs null).
fbst_status make_nulls(const fbst_plan* plan, int n, const int* qs, const double* u,
                       const double* v, bool interp, fbst_nulls** out) {
  const fbst::Params& p = plan->p;
  if (p.prec == FBST_PREC_FP64)
    return fail(FBST_E_UNSUPPORTED, "beamspace nulling takes complex64 data (not FBST_PREC_FP64)");
  const double gbytes = 8.0 * n * p.L * p.B * p.L;
  if (gbytes > 16.0 * (1ULL << 30))
    return fail(FBST_E_UNSUPPORTED, "the nulling tables would exceed 16 GiB");
  std::vector<double> uq(n), vq(n, 0.0);
  for (int i = 0; i < n; ++i) {
    if (qs) {
      uq[i] = p.u0 + (qs[i] / p.bv) * p.du;
      vq[i] = (p.kind != FBST_LINE) ? p.v0 + (qs[i] % p.bv) * p.dv : 0.0;
    } else {
      uq[i] = u[i];
      vq[i] = (v && p.kind != FBST_LINE) ? v[i] : 0.0;
    }
  }
  std::vector<fbst::zd> G, E;
  std::string msg;
  fbst_status s;
  try {
    s = fbst::build_null_tables(p, uq, vq, &G, (qs || interp) ? nullptr : &E, &msg);
  } catch (const std::bad_alloc&) {
    s = FBST_E_NOMEM;
    msg = "host allocation of the nulling tables failed";
  }
  if (s != FBST_OK) return fail(s, msg);
  Upload up;
  size_t o_map = 0, o_e = 0;
  VIOffsets o_vi;
  if (qs) {
    up.blob.resize(align_up(sizeof(int) * n));
    std::memcpy(up.blob.data(), qs, sizeof(int) * n);
  } else if (interp) {
    s = add_vector_interp(plan, uq, vq, &up, &o_vi);
    if (s != FBST_OK) return s;
  } else {
    o_e = up.add(E, false);
  }
  const size_t o_g = up.add(G, false);
  fbst_nulls* nl = new (std::nothrow) fbst_nulls();
  if (!nl) return fail(FBST_E_NOMEM, "host allocation failed");
  hipError_t e = hipMalloc(&nl->dev, up.blob.size());
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete nl;
    return fail(FBST_E_NOMEM, "hipMalloc of the nulling tables failed");
  }
  e = hipMemcpy(nl->dev, up.blob.data(), up.blob.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(nl->dev);
    delete nl;
    return hip_fail(e, "hipMemcpy of the nulling tables");
  }
  const unsigned char* b = static_cast<const unsigned char*>(nl->dev);
  nl->plan = plan;
  nl->P = n;
  if (qs) nl->map = reinterpret_cast<const int*>(b + o_map);
  else if (interp) nl->vi = vector_interp_at(nl->dev, o_vi);
  else nl->E = b + o_e;
  nl->G = b + o_g;
  nl->dev_bytes = up.blob.size();
  *out = nl;
  return FBST_OK;
}

// FBST_FLAG_DEVICE_GENERATORS: the Levinson solves of build_tables' columns
// on the GPU (float64), then the host completes the stage-2 tables.
// x_b = A_b^{-1} e_0 for the device columns dc [B][L] (complex128) into dx on
// stream st by the plan's solver (the superfast doubling Schur algorithm with
// FBST_FLAG_SUPERFAST_GENERATORS, else Levinson), status [B] into ds, GPU
// time into *ms; returns after the solve has finished.
hipError_t device_generator_solve(const fbst::Params& p, const void* dc, void* dx, int* ds,
                                  hipStream_t st, float* ms) {
  const bool superfast = (p.flags & FBST_FLAG_SUPERFAST_GENERATORS) != 0;
  void *sscr = nullptr, *stw = nullptr;
  size_t sbytes = 0;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipError_t e = hipSuccess;
  if (superfast) {
    const std::vector<fbst::zd> tw = fbst::superfast_twiddles(p.L);
    sbytes = fbst::superfast_scratch_bytes(p.B, p.L, nullptr);
    e = hipMalloc(&sscr, sbytes);
    if (e == hipSuccess) e = hipMalloc(&stw, tw.size() * 16);
    if (e == hipSuccess) e = hipMemcpy(stw, tw.data(), tw.size() * 16, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  if (e == hipSuccess) e = hipEventRecord(t0, st);
  if (e == hipSuccess)
    e = superfast ? fbst::launch_superfast(dc, dx, ds, p.B, p.L, sscr, sbytes, stw, st)
                  : fbst::launch_levinson(dc, dx, ds, p.B, p.L, st);
  if (e == hipSuccess) e = hipEventRecord(t1, st);
  if (e == hipSuccess) e = hipEventSynchronize(t1);
  *ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(ms, t0, t1);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  if (sscr) (void)hipFree(sscr);
  if (stw) (void)hipFree(stw);
  return e;
}

fbst_status solve_generators_on_device(fbst_plan* pl) {
  const fbst::Params& p = pl->p;
  const size_t n = static_cast<size_t>(p.B) * p.L;
  void *dc = nullptr, *dx = nullptr, *ds = nullptr;
  auto release = [&] {
    if (dc) (void)hipFree(dc);
    if (dx) (void)hipFree(dx);
    if (ds) (void)hipFree(ds);
  };
  if (hipMalloc(&dc, n * 16) != hipSuccess || hipMalloc(&dx, n * 16) != hipSuccess ||
      hipMalloc(&ds, sizeof(int) * p.B) != hipSuccess) {
    (void)hipGetLastError();
    release();
    return fail(FBST_E_NOMEM, "hipMalloc for the device generator solve failed");
  }
  std::vector<fbst::zd> x(n);
  std::vector<int> status(p.B, 1);
  hipError_t e = hipMemcpy(dc, pl->host.cols.data(), n * 16, hipMemcpyHostToDevice);
  float ms = 0.0f;
  if (e == hipSuccess) e = device_generator_solve(p, dc, dx, static_cast<int*>(ds), nullptr, &ms);
  pl->generator_ms = ms;
  if (e == hipSuccess) e = hipMemcpy(x.data(), dx, n * 16, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(status.data(), ds, sizeof(int) * p.B, hipMemcpyDeviceToHost);
  release();
  if (e != hipSuccess) return hip_fail(e, "device generator solve");
  for (int b = 0; b < p.B; ++b)
    if (status[b])
      return fail(FBST_E_INVALID, "Toeplitz system not positive definite in float64 (delta too small?)");
  if (fbst::finish_generators(p, x, pl->kept, &pl->host) != FBST_OK)
    return fail(FBST_E_INVALID, "device generator solve: inconsistent tables");
  return FBST_OK;
}

}  // namespace

extern "C" {

fbst_status fbst_plan_create(int M, int N, int B, const fbst_geometry* geometry,
                             const fbst_band* band, const fbst_grid* grid,
                             const fbst_options* options, fbst_plan** out) {
  if (!out) return fail(FBST_E_INVALID, "out is NULL");
  *out = nullptr;
  std::string msg;
  fbst::Params p;
  fbst_status st = fbst::resolve_params(M, N, B, geometry, band, grid, options, &p, &msg);
  if (st != FBST_OK) return fail(st, msg);
  fbst_plan* pl = new (std::nothrow) fbst_plan();
  if (!pl) return fail(FBST_E_NOMEM, "host allocation of the plan failed");
  pl->p = p;
  pl->host_only = (p.flags & FBST_FLAG_HOST_ONLY) != 0;
  pl->kept = pl->host_only || (p.flags & FBST_FLAG_KEEP_HOST_TABLES) != 0;
  pl->ws_bytes_per_block = ws_per_block(p);
  pl->ws_fixed_bytes = split_stage2(p) ? align_up(fbst::split_scratch_bytes(p.p3, true)) : 0;
  // stage 2 in the single-buffer form where it is compiled: at the same two
  // waves per SIMD it needs fewer registers than the dual form and runs
  // faster (fbst_autotune_ex measures all instances)
  if (!(p.flags & (FBST_FLAG_PRECOMPUTE | FBST_FLAG_STAGE2_REFINE)) &&
      fbst::k3_variant_available(p.p3, fp32_stage2(p), 1))
    pl->k3_variant.store(1);
  try {
    st = fbst::build_tables(p, pl->kept, &pl->host, &msg);
  } catch (const std::bad_alloc&) {
    st = FBST_E_NOMEM;
    msg = "host allocation of the plan tables failed";
  }
  if (st != FBST_OK) {
    delete pl;
    return fail(st, msg);
  }
  pl->nu_lanes = pl->host.nu_lanes;
  if (!pl->host_only && (p.flags & FBST_FLAG_DEVICE_GENERATORS)) {
    try {
      st = solve_generators_on_device(pl);
    } catch (const std::bad_alloc&) {
      st = fail(FBST_E_NOMEM, "host allocation of the generator tables failed");
    }
    if (st != FBST_OK) {
      delete pl;
      return st;
    }
  }
  if (!pl->host_only) {
    st = upload(pl);
    if (st != FBST_OK) {
      delete pl;
      return st;
    }
    if (p.flags & FBST_FLAG_PRECOMPUTE) {
      st = build_precomputed(pl);
      if (st != FBST_OK) {
        (void)hipFree(pl->dev);
        delete pl;
        return st;
      }
    }
    // device copies are the working set; keep only what was asked for on the host
    if (!pl->kept) pl->host = fbst::HostTables();
  }
  *out = pl;
  return FBST_OK;
}

fbst_status fbst_execute(const fbst_plan* plan, const void* x, void* beams, void* workspace,
                         void* hip_stream) {
  fbst_status s = check_exec(plan);
  if (s != FBST_OK) return s;
  if (!x || !beams) return fail(FBST_E_INVALID, "x and beams must not be NULL");
  void* ws = workspace ? workspace : plan->own_ws;
  hipError_t e = fbst::run_contiguous(plan, 1, 1, x, beams, ws, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "fbst_execute launch");
  return FBST_OK;
}

fbst_status fbst_execute_batched(const fbst_plan* plan, int nblocks, int max_chunk, const void* x,
                                 void* beams, void* workspace, void* hip_stream) {
  fbst_status s = check_exec(plan);
  if (s != FBST_OK) return s;
  if (nblocks < 0) return fail(FBST_E_INVALID, "nblocks must be >= 0");
  if (nblocks == 0) return FBST_OK;
  if (!x || !beams) return fail(FBST_E_INVALID, "x and beams must not be NULL");
  int chunk = (max_chunk <= 0 || max_chunk > nblocks) ? nblocks : max_chunk;
  if (chunk > fbst::MAX_LAUNCH_BLOCKS) chunk = fbst::MAX_LAUNCH_BLOCKS;
  void* ws = workspace;
  if (!ws) {
    if (chunk != 1) return fail(FBST_E_INVALID, "workspace is NULL but chunk > 1");
    ws = plan->own_ws;
  }
  hipError_t e = fbst::run_contiguous(plan, nblocks, chunk, x, beams, ws,
                                      static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "fbst_execute_batched launch");
  return FBST_OK;
}

fbst_status fbst_execute_stream(const fbst_plan* plan, long long T, int hop, const void* x,
                                void* beams, void* workspace, int max_chunk, void* hip_stream) {
  fbst_status s = check_exec(plan);
  if (s != FBST_OK) return s;
  const fbst::Params& p = plan->p;
  if (T < p.N || hop < 1) return fail(FBST_E_INVALID, "need T >= N and hop >= 1");
  if (!x || !beams) return fail(FBST_E_INVALID, "x and beams must not be NULL");
  const long long nblocks_ll = (T - p.N) / hop + 1;
  if (nblocks_ll > 0x7fffffffLL) return fail(FBST_E_INVALID, "too many windows");
  const int nblocks = static_cast<int>(nblocks_ll);
  int chunk = (max_chunk <= 0 || max_chunk > nblocks) ? nblocks : max_chunk;
  if (chunk > fbst::MAX_LAUNCH_BLOCKS) chunk = fbst::MAX_LAUNCH_BLOCKS;
  void* ws = workspace;
  if (!ws) {
    if (chunk != 1) return fail(FBST_E_INVALID, "workspace is NULL but chunk > 1");
    ws = plan->own_ws;
  }
  const size_t e = io_elem(p);
  const size_t out_blk = static_cast<size_t>(p.B) * p.N * e;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (int b0 = 0; b0 < nblocks; b0 += chunk) {
    const int n = (nblocks - b0 < chunk) ? nblocks - b0 : chunk;
    fbst::InPtrs xs{};
    fbst::OutPtrs outs{};
    xs.ld = T;
    for (int i = 0; i < n; ++i) {
      // window b0 + i starts at sample (b0 + i) hop of every sensor row
      xs.p[i] = static_cast<const unsigned char*>(x) + static_cast<size_t>(b0 + i) * hop * e;
      outs.p[i] = static_cast<unsigned char*>(beams) + (b0 + i) * out_blk;
    }
    const hipError_t he = fbst::run_blocks(plan, n, xs, outs, ws, st);
    if (he != hipSuccess) return hip_fail(he, "fbst_execute_stream launch");
  }
  return FBST_OK;
}

fbst_status fbst_execute_stage(const fbst_plan* plan, int stage, int nblocks, const void* in,
                               void* out, void* workspace, void* hip_stream) {
  fbst_status s = check_exec(plan);
  if (s != FBST_OK) return s;
  if (stage < 0 || stage > 2) return fail(FBST_E_INVALID, "stage must be 0, 1 or 2");
  if (nblocks < 1) return fail(FBST_E_INVALID, "nblocks must be >= 1");
  if (!in || !out) return fail(FBST_E_INVALID, "in and out must not be NULL");
  const fbst::Params& p = plan->p;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const size_t e1 = s1_elem(p), eio = io_elem(p);
  hipError_t e = hipSuccess;
  if (stage == 2 && plan->CA && !workspace) {
    // the refined stage 2 keeps beta_1 in the workspace
    if (nblocks != 1)
      return fail(FBST_E_INVALID, "the refined stage 2 over several blocks needs a workspace");
    workspace = plan->own_ws;
  }
  // the split float64 stage 2 needs ws_fixed_bytes of scratch, whatever nblocks
  if (stage == 2 && plan->ws_fixed_bytes && !workspace) workspace = plan->own_ws;
  if (stage == 1) {
    void* z = nullptr;
    if (p.kind != FBST_LINE) {
      if (!workspace) {
        if (nblocks != 1)
          return fail(FBST_E_INVALID, "stage 1 of a grid or arbitrary array over several blocks needs a workspace");
        workspace = plan->own_ws;
      }
      z = workspace;
    }
    e = stage1_double(p) ? run_stage1<double>(plan, nblocks, in, out, z, st)
                         : run_stage1<float>(plan, nblocks, in, out, z, st);
  } else {
    for (int b0 = 0; b0 < nblocks && e == hipSuccess; b0 += fbst::MAX_LAUNCH_BLOCKS) {
      const int n = std::min(fbst::MAX_LAUNCH_BLOCKS, nblocks - b0);
      if (stage == 0) {
        fbst::InPtrs xs{};
        for (int i = 0; i < n; ++i)
          xs.p[i] = static_cast<const unsigned char*>(in) + static_cast<size_t>(b0 + i) * p.M * p.N * eio;
        void* yh = static_cast<unsigned char*>(out) + static_cast<size_t>(b0) * p.M * p.L * e1;
        e = stage1_double(p) ? run_stage0<double>(plan, n, xs, yh, st) : run_stage0<float>(plan, n, xs, yh, st);
      } else {
        fbst::OutPtrs outs{};
        for (int i = 0; i < n; ++i)
          outs.p[i] = static_cast<unsigned char*>(out) + static_cast<size_t>(b0 + i) * p.B * p.N * eio;
        const void* w = static_cast<const unsigned char*>(in) + static_cast<size_t>(b0) * p.B * p.L * e1;
        e = run_stage2(plan, n, w, outs, workspace, st);
      }
    }
  }
  if (e != hipSuccess) return hip_fail(e, "fbst_execute_stage launch");
  return FBST_OK;
}

fbst_status fbst_graph_create(const fbst_plan* plan, int nblocks, int max_chunk, const void* x,
                              void* beams, void* workspace, fbst_graph** out) {
  if (!out) return fail(FBST_E_INVALID, "out is NULL");
  *out = nullptr;
  fbst_status s = check_exec(plan);
  if (s != FBST_OK) return s;
  if (nblocks < 1) return fail(FBST_E_INVALID, "nblocks must be >= 1");
  if (!x || !beams) return fail(FBST_E_INVALID, "x and beams must not be NULL");
  int chunk = (max_chunk <= 0 || max_chunk > nblocks) ? nblocks : max_chunk;
  if (chunk > fbst::MAX_LAUNCH_BLOCKS) chunk = fbst::MAX_LAUNCH_BLOCKS;
  void* ws = workspace;
  if (!ws) {
    if (chunk != 1) return fail(FBST_E_INVALID, "workspace is NULL but chunk > 1");
    ws = plan->own_ws;
  }
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "capture stream");
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    const hipError_t le = fbst::run_contiguous(plan, nblocks, chunk, x, beams, ws, cs);
    e = hipStreamEndCapture(cs, &graph);
    if (le != hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    if (exec) (void)hipGraphExecDestroy(exec);
    return hip_fail(e, "graph capture");
  }
  fbst_graph* g = new (std::nothrow) fbst_graph();
  if (!g) {
    (void)hipGraphExecDestroy(exec);
    return fail(FBST_E_NOMEM, "host allocation failed");
  }
  g->exec = exec;
  *out = g;
  return FBST_OK;
}

fbst_status fbst_graph_launch(const fbst_graph* graph, void* hip_stream) {
  if (!graph) return fail(FBST_E_INVALID, "graph is NULL");
  const hipError_t e = hipGraphLaunch(graph->exec, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return FBST_OK;
}

void fbst_graph_destroy(fbst_graph* graph) {
  if (!graph) return;
  (void)hipGraphExecDestroy(graph->exec);
  delete graph;
}

}  // extern "C"

namespace {

std::string device_arch(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  return prop.gcnArchName;
}

// Stage-2 variants the plan can launch (the refined and precomputed forms
// have one instance each).
std::vector<int> plan_variants(const fbst_plan* plan) {
  std::vector<int> v{0};
  const fbst::Params& p = plan->p;
  if (plan->K || plan->CA) return v;
  for (int var = 1; var <= 7; ++var)
    if (fbst::k3_variant_available(p.p3, fp32_stage2(p), var)) v.push_back(var);
  return v;
}

// Stage-1b workgroup sizes (variant bits 4-5) the plan can launch: the
// chirp-z of lines and grids in float32 has three.
std::vector<int> plan_tiles(const fbst_plan* plan) {
  const fbst::Params& p = plan->p;
  if (p.kind == FBST_ARBITRARY || stage1_double(p)) return {0};
  return {0, 1 << 4, 2 << 4};
}

// Every variant the plan accepts: a stage-2 variant with a stage-1b tile.
std::vector<int> plan_all_variants(const fbst_plan* plan) {
  std::vector<int> all;
  for (int t : plan_tiles(plan))
    for (int v : plan_variants(plan)) all.push_back(v | t);
  return all;
}

}  // namespace

extern "C" {

fbst_status fbst_plan_set_variant(const fbst_plan* plan, int variant) {
  fbst_status s = check_exec(plan);
  if (s != FBST_OK) return s;
  const std::vector<int> ok = plan_all_variants(plan);
  if (std::find(ok.begin(), ok.end(), variant) == ok.end())
    return fail(FBST_E_UNSUPPORTED, "stage-2 variant " + std::to_string(variant) +
                                        " is not compiled for this plan");
  const_cast<fbst_plan*>(plan)->k3_variant.store(variant);
  return FBST_OK;
}

int fbst_plan_variant(const fbst_plan* plan) { return plan ? plan->k3_variant.load() : -1; }

fbst_status fbst_autotune_ex(const fbst_plan* plan, int nblocks, const void* x, void* beams,
                             void* workspace, void* hip_stream, int force, int* best_chunk,
                             int* best_variant, float* best_ms) {
  fbst_status s = check_exec(plan);
  if (s != FBST_OK) return s;
  if (nblocks < 1 || !x || !beams || !workspace || !best_chunk)
    return fail(FBST_E_INVALID, "nblocks >= 1, x, beams, workspace and best_chunk are required");
  const fbst::Params& p = plan->p;
  const auto key = std::make_tuple(device_arch(plan->device), p.M, p.N, p.B, p.L,
                                   p.mx * 65536 + p.my, p.bu * 65536 + p.bv,
                                   static_cast<int>(p.prec), static_cast<int>(p.flags), nblocks,
                                   static_cast<int>(p.kind));
  struct Tuned {
    int chunk, variant;
    float ms;
  };
  static std::mutex mu;
  static std::map<decltype(key), Tuned> cache;
  fbst_plan* pl = const_cast<fbst_plan*>(plan);
  if (!force) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      pl->k3_variant.store(it->second.variant);
      *best_chunk = it->second.chunk;
      if (best_variant) *best_variant = it->second.variant;
      if (best_ms) *best_ms = it->second.ms;
      return FBST_OK;
    }
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const int before = pl->k3_variant.load();
  Tuned best{0, 0, 0.0f};
  for (int var : plan_variants(plan)) {
    pl->k3_variant.store(var);
    for (int chunk = 1; e == hipSuccess && chunk <= std::min(nblocks, fbst::MAX_LAUNCH_BLOCKS);
         chunk *= 2) {
      e = fbst::run_contiguous(plan, nblocks, chunk, x, beams, workspace, st);   // warm-up
      float acc = 0.0f;
      for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, st);
        if (e == hipSuccess) e = fbst::run_contiguous(plan, nblocks, chunk, x, beams, workspace, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        acc += ms;
      }
      const float ms = acc / 3.0f;
      if (e == hipSuccess && (best.chunk == 0 || ms < best.ms)) best = {chunk, var, ms};
    }
  }
  // then the stage-1b workgroup size at the chosen chunk and stage-2 variant
  const int chosen = best.variant;
  for (int t : plan_tiles(plan)) {
    if (t == 0 || e != hipSuccess) continue;
    pl->k3_variant.store(chosen | t);
    e = fbst::run_contiguous(plan, nblocks, best.chunk, x, beams, workspace, st);   // warm-up
    float acc = 0.0f;
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
      e = hipEventRecord(e0, st);
      if (e == hipSuccess) e = fbst::run_contiguous(plan, nblocks, best.chunk, x, beams, workspace, st);
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      acc += ms;
    }
    const float ms = acc / 3.0f;
    if (e == hipSuccess && ms < best.ms) best = {best.chunk, chosen | t, ms};
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) {
    pl->k3_variant.store(before);
    return hip_fail(e, "fbst_autotune");
  }
  pl->k3_variant.store(best.variant);
  {
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = best;
  }
  *best_chunk = best.chunk;
  if (best_variant) *best_variant = best.variant;
  if (best_ms) *best_ms = best.ms;
  return FBST_OK;
}

fbst_status fbst_autotune(const fbst_plan* plan, int nblocks, const void* x, void* beams,
                          void* workspace, void* hip_stream, int force, int* best_chunk,
                          float* best_ms) {
  return fbst_autotune_ex(plan, nblocks, x, beams, workspace, hip_stream, force, best_chunk,
                          nullptr, best_ms);
}

fbst_status fbst_nulls_create(const fbst_plan* plan, int n_interferers, const int* beams,
                              fbst_nulls** out) {
  if (!out) return fail(FBST_E_INVALID, "out is NULL");
  *out = nullptr;
  fbst_status s = check_exec(plan);
  if (s != FBST_OK) return s;
  if (n_interferers < 1 || n_interferers > 64 || !beams)
    return fail(FBST_E_INVALID, "need 1..64 interferer beams");
  const fbst::Params& p = plan->p;
  std::vector<int> qs(beams, beams + n_interferers);
  for (int q : qs)
    if (q < 0 || q >= p.B) return fail(FBST_E_INVALID, "interferer beam index out of range");
  return make_nulls(plan, n_interferers, qs.data(), nullptr, nullptr, false, out);
}

fbst_status fbst_nulls_create_directions(const fbst_plan* plan, int n_interferers, const double* u,
                                         const double* v, fbst_nulls** out) {
  if (!out) return fail(FBST_E_INVALID, "out is NULL");
  *out = nullptr;
  fbst_status s = check_exec(plan);
  if (s != FBST_OK) return s;
  if (n_interferers < 1 || n_interferers > 64 || !u)
    return fail(FBST_E_INVALID, "need 1..64 interferer directions");
  for (int i = 0; i < n_interferers; ++i)
    if (!std::isfinite(u[i]) || (v && !std::isfinite(v[i])))
      return fail(FBST_E_INVALID, "interferer directions must be finite");
  return make_nulls(plan, n_interferers, nullptr, u, v, false, out);
}

fbst_status fbst_nulls_create_interp(const fbst_plan* plan, int n_interferers, const double* u,
                                     const double* v, fbst_nulls** out) {
  if (!out) return fail(FBST_E_INVALID, "out is NULL");
  *out = nullptr;
  fbst_status s = check_exec(plan);
  if (s != FBST_OK) return s;
  if (n_interferers < 1 || n_interferers > 64 || !u)
    return fail(FBST_E_INVALID, "need 1..64 interferer directions");
  if (plan->p.bv > 1 && !v) return fail(FBST_E_INVALID, "a planar beam grid needs v");
  for (int i = 0; i < n_interferers; ++i)
    if (!std::isfinite(u[i]) || (v && !std::isfinite(v[i])))
      return fail(FBST_E_INVALID, "interferer directions must be finite");
  return make_nulls(plan, n_interferers, nullptr, u, v, true, out);
}

}  // extern "C"

namespace {

fbst_status make_directions(const fbst_plan* plan, int n_directions, const double* u,
                            const double* v, bool interp, fbst_directions** out) {
  if (!out) return fail(FBST_E_INVALID, "out is NULL");
  *out = nullptr;
  fbst_status s = check_exec(plan);
  if (s != FBST_OK) return s;
  const fbst::Params& p = plan->p;
  if (n_directions < 1 || n_directions > 65536 || !u)
    return fail(FBST_E_INVALID, "need 1..65536 directions");
  if (p.prec == FBST_PREC_FP64)
    return fail(FBST_E_UNSUPPORTED, "beams at directions take complex64 data (not FBST_PREC_FP64)");
  if (interp && p.bv > 1 && !v) return fail(FBST_E_INVALID, "a planar beam grid needs v");
  std::vector<double> ud(u, u + n_directions), vd(n_directions, 0.0);
  for (int i = 0; i < n_directions; ++i) {
    if (v && p.kind != FBST_LINE) vd[i] = v[i];
    if (!std::isfinite(ud[i]) || !std::isfinite(vd[i]))
      return fail(FBST_E_INVALID, "directions must be finite");
  }
  const double per_dir = 8.0 * p.L * (static_cast<double>(p.N) + (interp ? 0 : p.M));
  if (per_dir * n_directions > 16.0 * (1ULL << 30))
    return fail(FBST_E_UNSUPPORTED, "the direction tables would exceed 16 GiB");
  Upload up;
  VIOffsets o_vi;
  if (interp) {                                // validate the grid window first (cheap)
    s = add_vector_interp(plan, ud, vd, &up, &o_vi);
    if (s != FBST_OK) return s;
  }
  std::vector<fbst::zd> K, E;
  std::string msg;
  try {
    s = fbst::build_direction_tables(p, ud, vd, &K, interp ? nullptr : &E, &msg);
  } catch (const std::bad_alloc&) {
    s = FBST_E_NOMEM;
    msg = "host allocation of the direction tables failed";
  }
  if (s != FBST_OK) return fail(s, msg);
  const size_t o_e = interp ? 0 : up.add(E, false), o_k = up.add(K, false);
  fbst_directions* dr = new (std::nothrow) fbst_directions();
  if (!dr) return fail(FBST_E_NOMEM, "host allocation failed");
  hipError_t e = hipMalloc(&dr->dev, up.blob.size());
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete dr;
    return fail(FBST_E_NOMEM, "hipMalloc of the direction tables failed");
  }
  e = hipMemcpy(dr->dev, up.blob.data(), up.blob.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(dr->dev);
    delete dr;
    return hip_fail(e, "hipMemcpy of the direction tables");
  }
  const unsigned char* b = static_cast<const unsigned char*>(dr->dev);
  dr->plan = plan;
  dr->D = n_directions;
  if (interp) dr->vi = vector_interp_at(dr->dev, o_vi);
  else dr->E = b + o_e;
  dr->K = b + o_k;
  dr->dev_bytes = up.blob.size();
  *out = dr;
  return FBST_OK;
}

}  // namespace

extern "C" {

fbst_status fbst_directions_create(const fbst_plan* plan, int n_directions, const double* u,
                                   const double* v, fbst_directions** out) {
  return make_directions(plan, n_directions, u, v, false, out);
}

fbst_status fbst_directions_create_interp(const fbst_plan* plan, int n_directions,
                                          const double* u, const double* v,
                                          fbst_directions** out) {
  return make_directions(plan, n_directions, u, v, true, out);
}

void fbst_directions_destroy(fbst_directions* dirs) {
  if (!dirs) return;
  if (dirs->dev) (void)hipFree(dirs->dev);
  delete dirs;
}

size_t fbst_workspace_bytes_directions(const fbst_plan* plan, const fbst_directions* dirs,
                                       int nblocks) {
  if (!plan || !dirs || nblocks < 1) return 0;
  return directions_ws_per_block(plan, dirs) * static_cast<size_t>(nblocks);
}

fbst_status fbst_execute_directions(const fbst_plan* plan, const fbst_directions* dirs,
                                    int nblocks, int max_chunk, const void* x, void* beams,
                                    void* workspace, void* hip_stream) {
  fbst_status s = check_exec(plan);
  if (s != FBST_OK) return s;
  if (!dirs || dirs->plan != plan) return fail(FBST_E_INVALID, "directions were not made for this plan");
  if (nblocks < 0) return fail(FBST_E_INVALID, "nblocks must be >= 0");
  if (nblocks == 0) return FBST_OK;
  if (!x || !beams || !workspace) return fail(FBST_E_INVALID, "x, beams and workspace are required");
  int chunk = (max_chunk <= 0 || max_chunk > nblocks) ? nblocks : max_chunk;
  if (chunk > fbst::MAX_LAUNCH_BLOCKS) chunk = fbst::MAX_LAUNCH_BLOCKS;
  const fbst::Params& p = plan->p;
  const size_t in_blk = static_cast<size_t>(p.M) * p.N * 8;
  const size_t out_blk = static_cast<size_t>(dirs->D) * p.N * 8;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (int b0 = 0; b0 < nblocks; b0 += chunk) {
    const int n = (nblocks - b0 < chunk) ? nblocks - b0 : chunk;
    fbst::InPtrs xs{};
    for (int i = 0; i < n; ++i) xs.p[i] = static_cast<const unsigned char*>(x) + (b0 + i) * in_blk;
    const hipError_t e = run_blocks_directions(plan, dirs, n, xs,
                                               static_cast<unsigned char*>(beams) + b0 * out_blk,
                                               workspace, st);
    if (e != hipSuccess) return hip_fail(e, "fbst_execute_directions launch");
  }
  return FBST_OK;
}

fbst_status fbst_interp_create(const fbst_plan* plan, int n_directions, const double* u,
                               const double* v, fbst_interp** out) {
  if (!out) return fail(FBST_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!plan) return fail(FBST_E_INVALID, "plan is NULL");
  fbst_status s = FBST_OK;
  if (n_directions < 1 || n_directions > 65536 || !u)
    return fail(FBST_E_INVALID, "need 1..65536 directions");
  const bool plane = plan->p.bv > 1;
  if (plane && !v) return fail(FBST_E_INVALID, "a planar beam grid needs v");
  std::vector<double> ud(u, u + n_directions), vd(n_directions, 0.0);
  if (plane) vd.assign(v, v + n_directions);
  for (int i = 0; i < n_directions; ++i)
    if (!std::isfinite(ud[i]) || !std::isfinite(vd[i]))
      return fail(FBST_E_INVALID, "directions must be finite");
  fbst_interp* it = new (std::nothrow) fbst_interp();
  if (!it) return fail(FBST_E_NOMEM, "host allocation failed");
  std::string msg;
  try {
    s = fbst::build_interp_table(plan->p, ud, vd, &it->host_first, &it->host_w, &msg);
  } catch (const std::bad_alloc&) {
    s = FBST_E_NOMEM;
    msg = "host allocation of the interpolation table failed";
  }
  if (s != FBST_OK) {
    delete it;
    return fail(s, msg);
  }
  it->plan = plan;
  it->D = n_directions;
  if (plan->host_only) {                       // the host table only (no device memory)
    *out = it;
    return FBST_OK;
  }
  const size_t o_w = (it->host_first.size() * sizeof(int) + 255) / 256 * 256;
  const size_t bytes = o_w + it->host_w.size() * sizeof(double);
  hipError_t e = hipMalloc(&it->dev, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    delete it;
    return fail(FBST_E_NOMEM, "hipMalloc of the interpolation table failed");
  }
  unsigned char* b = static_cast<unsigned char*>(it->dev);
  e = hipMemcpy(b, it->host_first.data(), it->host_first.size() * sizeof(int),
                hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b + o_w, it->host_w.data(), it->host_w.size() * sizeof(double),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(it->dev);
    delete it;
    return hip_fail(e, "hipMemcpy of the interpolation table");
  }
  it->first = reinterpret_cast<const int*>(b);
  it->w = reinterpret_cast<const double*>(b + o_w);
  *out = it;
  return FBST_OK;
}

void fbst_interp_destroy(fbst_interp* interp) {
  if (!interp) return;
  if (interp->dev) (void)hipFree(interp->dev);
  delete interp;
}

fbst_status fbst_interp_table(const fbst_interp* interp, int* first, double* w) {
  if (!interp) return fail(FBST_E_INVALID, "interp is NULL");
  if (first) std::copy(interp->host_first.begin(), interp->host_first.end(), first);
  if (w) std::copy(interp->host_w.begin(), interp->host_w.end(), w);
  return FBST_OK;
}

fbst_status fbst_execute_interp(const fbst_interp* interp, int nblocks, const void* beams,
                                void* out, void* hip_stream) {
  if (!interp) return fail(FBST_E_INVALID, "interp is NULL");
  fbst_status s = check_exec(interp->plan);
  if (s != FBST_OK) return s;
  if (nblocks < 0) return fail(FBST_E_INVALID, "nblocks must be >= 0");
  if (nblocks == 0) return FBST_OK;
  if (!beams || !out) return fail(FBST_E_INVALID, "beams and out are required");
  const fbst::Params& p = interp->plan->p;
  const hipError_t e = fbst::launch_interp_beams(beams, interp->first, interp->w, out, p.B,
                                                 p.bv, interp->D, p.N, nblocks,
                                                 p.prec == FBST_PREC_FP64,
                                                 static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "fbst_execute_interp launch");
  return FBST_OK;
}

void fbst_nulls_destroy(fbst_nulls* nulls) {
  if (!nulls) return;
  if (nulls->dev) (void)hipFree(nulls->dev);
  delete nulls;
}

size_t fbst_workspace_bytes_nulled(const fbst_plan* plan, const fbst_nulls* nulls, int nblocks) {
  if (!plan || !nulls || nblocks < 1) return 0;
  return nulled_ws_per_block(plan, nulls) * static_cast<size_t>(nblocks) + plan->ws_fixed_bytes;
}

fbst_status fbst_execute_nulled(const fbst_plan* plan, const fbst_nulls* nulls, int nblocks,
                                int max_chunk, const void* x, void* beams, void* workspace,
                                void* hip_stream) {
  fbst_status s = check_exec(plan);
  if (s != FBST_OK) return s;
  if (!nulls || nulls->plan != plan) return fail(FBST_E_INVALID, "nulls were not made for this plan");
  if (nblocks < 0) return fail(FBST_E_INVALID, "nblocks must be >= 0");
  if (nblocks == 0) return FBST_OK;
  if (!x || !beams || !workspace) return fail(FBST_E_INVALID, "x, beams and workspace are required");
  int chunk = (max_chunk <= 0 || max_chunk > nblocks) ? nblocks : max_chunk;
  if (chunk > fbst::MAX_LAUNCH_BLOCKS) chunk = fbst::MAX_LAUNCH_BLOCKS;
  const fbst::Params& p = plan->p;
  const size_t in_blk = static_cast<size_t>(p.M) * p.N * 8, out_blk = static_cast<size_t>(p.B) * p.N * 8;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (int b0 = 0; b0 < nblocks; b0 += chunk) {
    const int n = (nblocks - b0 < chunk) ? nblocks - b0 : chunk;
    fbst::InPtrs xs{};
    fbst::OutPtrs outs{};
    for (int i = 0; i < n; ++i) {
      xs.p[i] = static_cast<const unsigned char*>(x) + (b0 + i) * in_blk;
      outs.p[i] = static_cast<unsigned char*>(beams) + (b0 + i) * out_blk;
    }
    const hipError_t e = run_blocks_nulled(plan, nulls, n, xs, outs, workspace, st);
    if (e != hipSuccess) return hip_fail(e, "fbst_execute_nulled launch");
  }
  return FBST_OK;
}

fbst_status fbst_plan_steer(fbst_plan* plan, const fbst_grid* grid, void* hip_stream) {
  fbst_status s = check_exec(plan);
  if (s != FBST_OK) return s;
  if (plan->K || plan->CA)
    return fail(FBST_E_UNSUPPORTED, "a new beam grid needs a plan without FBST_FLAG_PRECOMPUTE "
                                    "and FBST_FLAG_STAGE2_REFINE");
  fbst::Params q = plan->p;
  std::string msg;
  s = fbst::resolve_grid(&q, grid, &msg);
  if (s != FBST_OK) return fail(s, msg);
  if (q.bu != plan->p.bu || q.bv != plan->p.bv)
    return fail(FBST_E_INVALID, "the new beam grid must keep bu and bv");
  int device = -1;
  hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (device != plan->device) return fail(FBST_E_INVALID, "the plan's device must be the current device");
  fbst::HostTables t;
  fbst::SteerKeys keys;
  try {
    const bool refine_host = 2.0 * q.M * q.N / q.delta > 1e6;
    s = fbst::build_steer_tables(q, &t, &keys, refine_host || plan->kept, &msg);
  } catch (const std::bad_alloc&) {
    return fail(FBST_E_NOMEM, "host allocation of the steering tables failed");
  }
  if (s != FBST_OK) return fail(s, msg);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // launches already issued on the stream still read the old tables
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  // one real centred system per distinct (|u|, |v|), as at plan creation
  fbst::Params qk = q;
  qk.B = static_cast<int>(keys.rcols.size() / q.L);
  const size_t nk = keys.rcols.size();
  void *dc = nullptr, *dx = nullptr, *ds = nullptr, *dtw = nullptr, *dkey = nullptr, *dsb = nullptr;
  auto release = [&] {
    for (void* ptr : {dc, dx, ds, dtw, dkey, dsb})
      if (ptr) (void)hipFree(ptr);
  };
  if (hipMalloc(&dc, nk * 16) != hipSuccess || hipMalloc(&dx, nk * 16) != hipSuccess ||
      hipMalloc(&ds, sizeof(int) * qk.B) != hipSuccess) {
    (void)hipGetLastError();
    release();
    return fail(FBST_E_NOMEM, "hipMalloc for the steering solve failed");
  }
  std::vector<int> status(qk.B, 1);
  float ms = 0.0f;
  e = hipMemcpy(dc, keys.rcols.data(), nk * 16, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = device_generator_solve(qk, dc, dx, static_cast<int*>(ds), st, &ms);
  if (e == hipSuccess) e = hipMemcpy(status.data(), ds, sizeof(int) * qk.B, hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    release();
    return hip_fail(e, "steering generator solve");
  }
  for (int k = 0; k < qk.B; ++k)
    if (status[k]) {
      release();
      return fail(FBST_E_INVALID, "Toeplitz system not positive definite in float64 (delta too small?)");
    }
  // Nothing of the plan has changed so far.  Spectra: on the device, or,
  // when cond(A) calls for refinement (as in build_tables), refined and
  // transformed on the host; kept host tables are refreshed on the host.
  const bool refine = 2.0 * q.M * q.N / q.delta > 1e6;
  const bool d1 = stage1_double(q), d2 = stage2_double(q);
  const size_t n = static_cast<size_t>(q.B) * q.L;
  const size_t gbytes = static_cast<size_t>(q.B) * q.p3 * (d2 ? 16 : 8);
  Upload up;
  if (refine || plan->kept) {
    std::vector<fbst::zd> xk(nk), x(n);
    e = hipMemcpy(xk.data(), dx, nk * 16, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      release();
      return hip_fail(e, "steering generator download");
    }
    try {
      for (int b = 0; b < q.B; ++b) {
        const fbst::zd* r = xk.data() + static_cast<size_t>(keys.key[b]) * q.L;
        fbst::zd* xb = x.data() + static_cast<size_t>(b) * q.L;
        for (int d = 0; d < q.L; ++d)
          xb[d] = std::polar(1.0, -2.0 * 3.141592653589793238 * q.eps * d / q.L * keys.s[b]) *
                  r[d].real();
        xb[0] = fbst::zd(r[0].real(), 0.0);
      }
      t.G1.assign(static_cast<size_t>(q.B) * q.p3, fbst::zd());
      t.G2.assign(static_cast<size_t>(q.B) * q.p3, fbst::zd());
      if (plan->kept) {
        t.gram.assign(n, fbst::zd());
        t.gen.assign(n, fbst::zd());
      }
      if (fbst::finish_generators(q, x, plan->kept, &t) != FBST_OK) {
        release();
        return fail(FBST_E_INVALID, "steering: inconsistent tables");
      }
    } catch (const std::bad_alloc&) {
      release();
      return fail(FBST_E_NOMEM, "host allocation of the steering spectra failed");
    }
  }
  if (refine) {
    const size_t o1 = up.add(t.G1, d2), o2 = up.add(t.G2, d2);
    e = hipMemcpy(const_cast<void*>(plan->G1), up.blob.data() + o1, gbytes, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(const_cast<void*>(plan->G2), up.blob.data() + o2, gbytes, hipMemcpyHostToDevice);
  } else {
    const std::vector<fbst::zd> tw = twiddles();
    e = hipMalloc(&dtw, tw.size() * 16);
    if (e == hipSuccess) e = hipMalloc(&dkey, sizeof(int) * q.B);
    if (e == hipSuccess) e = hipMalloc(&dsb, sizeof(double) * q.B);
    if (e == hipSuccess) e = hipMemcpy(dtw, tw.data(), tw.size() * 16, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(dkey, keys.key.data(), sizeof(int) * q.B, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dsb, keys.s.data(), sizeof(double) * q.B, hipMemcpyHostToDevice);
    void* g1 = const_cast<void*>(plan->G1);
    void* g2 = const_cast<void*>(plan->G2);
    const int* kp = static_cast<const int*>(dkey);
    const double* sp = static_cast<const double*>(dsb);
    if (e == hipSuccess)
      e = d2 ? fbst::launch_gs_spectra<double>(q.p3, dx, q.B, q.L, g1, g2, dtw, st, kp, sp, q.eps)
             : fbst::launch_gs_spectra<float>(q.p3, dx, q.B, q.L, g1, g2, dtw, st, kp, sp, q.eps);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  // stage-1b chirps of the new grid, in place of the old
  if (e == hipSuccess) {
    Upload ax;
    const size_t a0 = ax.add(t.ax.pre, d1), a1 = ax.add(t.ax.H, d1), a2 = ax.add(t.ax.post, d1);
    const size_t el = d1 ? 16 : 8;
    e = hipMemcpy(const_cast<void*>(plan->axp), ax.blob.data() + a0, t.ax.pre.size() * el, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(const_cast<void*>(plan->axH), ax.blob.data() + a1, t.ax.H.size() * el, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(const_cast<void*>(plan->axq), ax.blob.data() + a2, t.ax.post.size() * el, hipMemcpyHostToDevice);
    if (e == hipSuccess && q.kind == FBST_GRID) {
      Upload ay;
      const size_t b0 = ay.add(t.ay.pre, d1), b1 = ay.add(t.ay.H, d1), b2 = ay.add(t.ay.post, d1);
      e = hipMemcpy(const_cast<void*>(plan->ayp), ay.blob.data() + b0, t.ay.pre.size() * el, hipMemcpyHostToDevice);
      if (e == hipSuccess)
        e = hipMemcpy(const_cast<void*>(plan->ayH), ay.blob.data() + b1, t.ay.H.size() * el, hipMemcpyHostToDevice);
      if (e == hipSuccess)
        e = hipMemcpy(const_cast<void*>(plan->ayq), ay.blob.data() + b2, t.ay.post.size() * el, hipMemcpyHostToDevice);
    }
  }
  release();
  // the plan now describes the new grid (also when an upload failed part-way:
  // its tables are then mixed, and the error says so)
  plan->p = q;
  plan->generator_ms = ms;
  if (plan->kept) {
    fbst::HostTables& h = plan->host;
    h.ax = std::move(t.ax);
    h.ay = std::move(t.ay);
    h.u = std::move(t.u);
    h.v = std::move(t.v);
    h.G1 = std::move(t.G1);
    h.G2 = std::move(t.G2);
    h.gram = std::move(t.gram);
    h.gen = std::move(t.gen);
  }
  if (e != hipSuccess) return hip_fail(e, "steering table upload (the plan's tables are inconsistent)");
  return FBST_OK;
}

size_t fbst_workspace_bytes(const fbst_plan* plan, int nblocks) {
  if (!plan || nblocks < 1) return 0;
  return plan->ws_bytes_per_block * static_cast<size_t>(nblocks) + plan->ws_fixed_bytes;
}

size_t fbst_plan_device_bytes(const fbst_plan* plan) { return plan ? plan->dev_bytes : 0; }

fbst_status fbst_plan_info(const fbst_plan* plan, fbst_info* info) {
  if (!plan || !info) return fail(FBST_E_INVALID, "plan and info must not be NULL");
  const fbst::Params& p = plan->p;
  info->M = p.M;
  info->N = p.N;
  info->B = p.B;
  info->L = p.L;
  info->mx = p.mx;
  info->my = p.my;
  info->bu = p.bu;
  info->bv = p.bv;
  info->p1 = p.p1;
  info->p2x = p.p2x;
  info->p2y = p.p2y;
  info->p3 = p.p3;
  info->precision = p.prec;
  info->io_elem_bytes = (p.prec == FBST_PREC_FP64) ? 16 : 8;
  info->device_bytes = plan->dev_bytes;
  info->workspace_per_block = plan->ws_bytes_per_block;
  info->generator_ms = plan->generator_ms;
  info->workspace_fixed = plan->ws_fixed_bytes;
  info->p1_split = p.p1s;
  info->stage2_precomputed = plan->K ? 1 : 0;
  info->nu_width = p.nuw;
  info->nu_lanes = (p.kind == FBST_ARBITRARY && !p.p2y) ? plan->nu_lanes : 0;
  info->cond_bound = p.cond_bound;
  return FBST_OK;
}

fbst_status fbst_plan_table(const fbst_plan* plan, int table, void* dst, size_t bytes) {
  if (!plan || !dst) return fail(FBST_E_INVALID, "plan and dst must not be NULL");
  if (!plan->kept) return fail(FBST_E_INVALID, "host tables were not kept for this plan");
  const fbst::HostTables& h = plan->host;
  const void* src = nullptr;
  size_t need = 0;
  switch (table) {
    case FBST_TABLE_BEAM_U:
      src = h.u.data();
      need = h.u.size() * sizeof(double);
      break;
    case FBST_TABLE_BEAM_V:
      src = h.v.data();
      need = h.v.size() * sizeof(double);
      break;
    case FBST_TABLE_GRAM:
      src = h.gram.data();
      need = h.gram.size() * sizeof(fbst::zd);
      break;
    case FBST_TABLE_GENERATOR:
      src = h.gen.data();
      need = h.gen.size() * sizeof(fbst::zd);
      break;
    default:
      return fail(FBST_E_INVALID, "unknown table id");
  }
  if (need == 0) return fail(FBST_E_INVALID, "table is empty");
  if (bytes < need) return fail(FBST_E_INVALID, "destination too small");
  std::memcpy(dst, src, need);
  return FBST_OK;
}

void fbst_destroy(fbst_plan* plan) {
  if (!plan) return;
  if (plan->dev) (void)hipFree(plan->dev);
  if (plan->K) (void)hipFree(plan->K);
  delete plan;
}

const char* fbst_last_error(void) { return g_last_error.c_str(); }

const char* fbst_version(void) { return "fbst-gfx950 0.1"; }

}  // extern "C"
