// Host-side launchers of the FBST kernels (kernels.hip).  Pointers are device
// pointers to interleaved complex arrays of the template element type; P is
// the FFT size of the launch (power of two, 32..16384; 8192 at most for
// double); tw is the twiddle array of fft_lds.h (TW_TABLE entries).  All
// return the HIP error of the launch.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/fbst.h"
#include "cx.h"

namespace fbst {

// Blocks of one launch: each block's input (or output) buffer is given by its
// own pointer, passed by value in the kernel arguments, so one launch can
// serve blocks that live anywhere (a contiguous batch or separate requests).
constexpr int MAX_LAUNCH_BLOCKS = FBST_MAX_LAUNCH_BLOCKS;
struct InPtrs {
  const void* p[MAX_LAUNCH_BLOCKS];
  long long ld = 0;    // elements between consecutive sensor rows of x (0: N, a [M][N] block)
};
struct OutPtrs {
  void* p[MAX_LAUNCH_BLOCKS];
};

// Stage 1a: yhat[blk][m][i] = sum_n x_blk[m][n] exp(-j omega_{i+1} t_n), blk < nblocks.
template <typename T>
hipError_t launch_time_czt(int P, const InPtrs& xs, int nblocks, void* yhat, const void* pre,
                           const void* H, const void* post, const void* tw, int M, int N, int L,
                           hipStream_t st);

// Stage 1a in split-output form: outputs [0, Ls) and [Ls, L) from two
// P-point convolutions sharing one forward FFT (P >= N + Ls - 1, L - Ls <= Ls);
// Ha, Hb are the kernel spectra of the two halves.
template <typename T>
hipError_t launch_time_czt_split(int P, const InPtrs& xs, int nblocks, void* yhat, const void* pre,
                                 const void* Ha, const void* Hb, const void* post, const void* tw,
                                 int M, int N, int L, int Ls, hipStream_t st);

// Stage 1a on the matrix cores (bfloat16, or float16 when fp16), split
// precision with float32 accumulation; complex64 in and out; P in
// {1024, 2048, 4096, 8192, 16384}.
hipError_t launch_time_czt_mfma(int P, bool fp16, const InPtrs& xs, int nblocks, void* yhat,
                                const void* pre, const void* H, const void* post, const void* tw,
                                int M, int N, int L, hipStream_t st);

// Stage 1b, one axis: layout [nb][pre_n][A][post_n][L], A = a_in -> a_out.
// tile: workgroup size of the instance (frequencies per workgroup): 0 the
// default, 1 half, 2 twice (float32 only; else hipErrorInvalidValue).
template <typename T>
hipError_t launch_axis_czt(int P, const void* in, void* out, const void* pre, const void* H,
                           const void* post, const void* tw, int a_in, int a_out, int pre_n,
                           int post_n, int L, int nblocks, hipStream_t st, int tile = 0);

// Stage 1b for arbitrary positions (type-1 non-uniform FFT per frequency):
// spread yhat [nb][M][L] onto the oversampled grid out [nb][nfx][nfy][L]
// (width W = 8 for float, 16 for double; tables [M][L]; posy only when
// nfy > 1; for nfy = 1, lanes elements per frequency at once in the element
// order given, whose supports the caller has checked to be disjoint),
// then per axis an nf-point FFT and the modes a - a_out/2 scaled by corr[a]
// (layout [nb][pre_n][P][post_n][L] -> [nb][pre_n][a_out][post_n][L]).
template <typename T>
hipError_t launch_nu_spread(int width, const void* in, void* out, const void* pre, const void* posx,
                            const void* posy, const int* order, int lanes, int M, int nfx, int nfy,
                            double beta, int L, int nblocks, hipStream_t st);
// Line of beams, spread + FFT + modes in one kernel (oversampled grid of
// P = 256..4096 points kept in LDS): yhat [nb][M][L] -> w [nb][a_out][L].
// hipErrorInvalidValue for other P (the caller then uses the two-kernel path).
template <typename T>
hipError_t launch_nu_line_fused(int width, int P, const void* in, void* w, const void* pre,
                                const void* pos, const int* order, int lanes, const void* corr,
                                const void* tw, int M, int a_out, double beta, int L, int nblocks,
                                hipStream_t st);
// 2-D beam grid, spread + row and column FFTs + modes in one kernel (32 x 32
// oversampled grid, beam grids up to 16 x 16): yhat -> w [nb][bu bv][L].
template <typename T>
hipError_t launch_nu_plane_fused(int width, int nfx, int nfy, const void* in, void* w,
                                 const void* pre, const void* posx, const void* posy,
                                 const void* cxs, const void* cys, const void* tw, int M, int bu,
                                 int bv, double beta, int L, int nblocks, hipStream_t st);
template <typename T>
hipError_t launch_axis_dft(int P, const void* in, void* out, const void* corr, const void* tw,
                           int a_out, int pre_n, int post_n, int L, int nblocks, hipStream_t st);

// Stage 2: beams_blk[b][n] from w[blk][b][0..L-1], blk < nblocks; needs 2L <= P.
// var selects a compiled instance (bit 0: the two Gohberg-Semencul branches in
// sequence in one LDS buffer instead of as one dual transform; bit 1: a
// persistent grid of the resident workgroups, each taking a contiguous range
// of rows); bit 1 leaves the beams bit-identical, bit 0 changes them at the
// level of float32 rounding.  Variants other than 0
// exist for a float32 stage 2 at P >= 1024 (k3_variant_available), else
// hipErrorInvalidValue.
template <typename T, typename TIN, typename TOUT>
hipError_t launch_toeplitz_fu(int P, const void* w, const OutPtrs& outs, const void* G1,
                              const void* G2, const void* pre3, const void* H3, const void* post3,
                              const void* tw, int B, int L, int N, int nblocks, hipStream_t st,
                              int var = 0);
bool k3_variant_available(int P, bool fp32_stage2, int var);

// Stage 2 in float64 at P = 8192 or 16384 with every P-point transform split
// into two P/2-point transforms in LDS (the form for P = 16384, where one
// float64 transform exceeds the LDS).  scratch: split_scratch_bytes(P) bytes
// of device memory, overwritten.  Needs 2L <= P and N + L - 1 <= P.
size_t split_scratch_bytes(int P, bool dbl);   // dbl: float64 stage 2
template <typename T, typename TIN, typename TOUT>
hipError_t launch_toeplitz_fu_split(int P, const void* w, const OutPtrs& outs, const void* G1,
                                    const void* G2, const void* pre3, const void* H3,
                                    const void* post3, const void* tw, void* scratch, int B, int L,
                                    int N, int nblocks, hipStream_t st);

// Stage 2 in float32 with one step of iterative refinement: beta_1 = A^{-1} w
// by Gohberg-Semencul (stored to bt [nblocks][B][L]), then beta = beta_1 +
// A^{-1} (w - A beta_1) with A applied through its circulant-embedding
// spectrum CA [B][P] (already divided by P), then F_u; two launches.
hipError_t launch_toeplitz_fu_refined(int P, const void* w, const OutPtrs& outs, const void* G1,
                                      const void* G2, const void* pre3, const void* H3,
                                      const void* post3, const void* tw, const void* CA, void* bt,
                                      int B, int L, int N, int nblocks, hipStream_t st);

// Per-group complex product over the blocks of a launch (complex64):
//   out[blk][g][n] = sum_k K[k][g][n] in[blk][row(g)][k]        (g < NG, n < NO, k < KL)
// row(g) = in_map[g] (a device array) if given, else 0 when in_rows == 1, else g;
// the input of block blk is the rows in[blk * in_rows ... ][KL].  The result
// goes to out [nb][NG][NO] when out is given, else to outs.p[blk] + g NO; with
// base ([nb][NG][NO]) the stored value is base - product.
struct ProductArgs {
  const cx<float>* K = nullptr;
  const cx<float>* in = nullptr;
  const int* in_map = nullptr;
  int in_rows = 1;
  OutPtrs outs{};
  cx<float>* out = nullptr;
  const cx<float>* base = nullptr;
  int NG = 0, KL = 0, NO = 0, nb = 0;
};
hipError_t launch_beam_product(const ProductArgs& a, hipStream_t st);

// Stage 2 in precomputed form: beams_blk[b][n] = sum_l K[l][b][n] w[blk][b][l]
// (complex64, K = F_u A_b^{-1} per beam stored [L][B][N]) on the float32
// matrix cores.
hipError_t launch_precomputed_apply(const void* K, const void* w, const OutPtrs& outs, int B,
                                    int L, int N, int nblocks, hipStream_t st);

// out[blk][q][l] = w[blk][map[q]][l] (complex64; map: P device ints).
hipError_t launch_gather_rows(const void* w, const int* map, void* out, int B, int P, int L,
                              int nblocks, hipStream_t st);

// out[blk][q][l] = sum_m yhat[blk][m][l] E[q][m][l] (complex64; yhat [nb][M][L],
// E [P][M][L]).
hipError_t launch_project_dirs(const void* yhat, const void* E, void* out, int M, int P, int L,
                               int nblocks, hipStream_t st);

// x [B][L] = first columns of the inverses of the Hermitian Toeplitz matrices
// with first columns cols [B][L] (complex128), Levinson recursion in float64,
// L <= 8192; status [B] (device ints): 0, or 1 if a pivot is not positive.
hipError_t launch_levinson(const void* cols, void* x, int* status, int B, int L, hipStream_t st);

// Spectra of the Gohberg-Semencul factors from generators x [B][L]
// (complex128): G1[b] = FFT_P(x_b) s_b, G2[b] = FFT_P(y~_b) s_b with
// s_b = 1 / (P sqrt(x_b[0])) and y~_b = (0, conj x_b[L-1], ..., conj x_b[1]),
// computed in float64 and stored [B][P] in TG (float or double); tw64: the
// per-pass twiddle tables in float64.  With key (device int [B]) and s
// (device double [B]), x holds generators of real centred systems [K][L] and
// beam b's is x[key[b]][d] exp(-j 2 pi eps d s[b] / L).  Needs 2L <= P <= PMAX.
template <typename TG>
hipError_t launch_gs_spectra(int P, const void* x, int B, int L, void* G1, void* G2,
                             const void* tw64, hipStream_t st, const int* key = nullptr,
                             const double* s = nullptr, double eps = 0.0);

// The same x [B][L] by the superfast doubling Schur algorithm (superfast.h),
// float64, one workgroup per system, L <= 4096.  scratch: device memory of at
// least superfast_scratch_bytes(B, L) bytes (grid: the workgroups launched);
// tw: superfast_twiddles(L) (complex128, max_fft(L) / 2 entries).
size_t superfast_scratch_bytes(int B, int L, int* grid);
hipError_t launch_superfast(const void* cols, void* x, int* status, int B, int L, void* scratch,
                            size_t scratch_bytes, const void* tw, hipStream_t st);

// out[blk][d][n] = sum_{i<8, j<TV} wu[d][i] wv[d][j] beams[blk][(a0 + i) bv + c0 + j][n]
// with (a0, c0) = first[d] and (wu, wv) = w[d] (TV = 8 if bv > 1, else 1);
// complex64, or complex128 when fp64; beams [nb][B][N], out [nb][D][N];
// first and w are device arrays [D][2] and [D][2][8].
hipError_t launch_interp_beams(const void* beams, const int* first, const double* w, void* out,
                               int B, int bv, int D, int N, int nblocks, bool fp64,
                               hipStream_t st);

// Beamspace vectors interpolated at directions with the reference point at
// the array's centre: out[blk][d][l] = sum_{i<8, j<TV} wu[d][i] wv[d][j]
// exp(j (theta[l] (fu - i) + theta[L + l] (fv - j))) W[blk][(a0 + i) bv + c0 + j][l]
// ((a0, c0) = first[d], (fu, fv) = frac[d]); complex64, W [nb][B][L],
// out [nb][D][L]; first [D][2], w [D][2][8], frac [D][2], theta [2][L] on
// the device.
hipError_t launch_interp_vectors(const void* W, const int* first, const double* w,
                                 const double* frac, const double* theta, void* out, int B,
                                 int bv, int D, int L, int nblocks, hipStream_t st);

// w[j][b][l] = (l == l0 + j) for j < rows (complex64, [rows][B][L]).
hipError_t launch_unit_rows(void* w, int B, int L, int l0, int rows, hipStream_t st);

}  // namespace fbst
