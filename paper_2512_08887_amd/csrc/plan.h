// Plan object and FP64 host table builder of the FBST library.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <complex>
#include <cstddef>
#include <string>
#include <vector>

#include "../../include/fbst.h"

namespace fbst {

using zd = std::complex<double>;

// One axis of the stage-1b spatial chirp-z (Sec. IV; App. B per axis):
// out[a] = sum_i in[i] exp(j rho_l u_a pos_i), pos_i = (o + i) d samples,
// u_a = u0 + a du.  Tables are l-fastest: pre [a_in][L], H [P][L], post [a_out][L].
struct AxisTables {
  int a_in = 0, a_out = 0, P = 0;
  std::vector<zd> pre, H, post;
};

struct HostTables {
  std::vector<zd> pre1, H1, post1;        // stage 1a: [N], [P1], [L]
  std::vector<zd> H1a, H1b;               // split-output stage 1a: [P1s] per output half
  AxisTables ax, ay;                      // stage 1b (ay unused for a line)
  std::vector<zd> G1, G2;                 // stage 2: [B][P3] spectra of x_b and y~_b
  std::vector<zd> CA;                     // FBST_FLAG_STAGE2_REFINE: [B][P3] spectrum of the
                                          // circulant embedding of A_b, divided by P3
  std::vector<zd> pre3, H3, post3;        // F_u chirp-z: [L], [P3], [N]
  std::vector<double> u, v;               // beam direction cosines [B]
  std::vector<zd> gram, gen;              // [B][L] (kept on request)
  // non-uniform stage 1b (arbitrary positions): centre-direction phases
  // nu_pre [M][L]; per axis the spreading position of element m at frequency l
  // as (f, j0) [M][L] (first grid point j0 of the kernel support, fractional
  // offset f in [0, 1) of the point beyond grid point j0 + w/2 - 1); and the
  // deconvolution factors per output mode, nu_cx [bu], nu_cy [bv] (real).
  std::vector<zd> nu_pre, nu_posx, nu_posy, nu_cx, nu_cy;
  // line of beams: elements in increasing x (nu_order [M]) and the lanes per
  // frequency of the spread (each lane takes a contiguous run of that order;
  // the runs' elements taken together never share a grid cell)
  std::vector<int> nu_order;
  int nu_lanes = 1;
  // FBST_FLAG_DEVICE_GENERATORS: Toeplitz first columns [B][L] (with delta)
  // awaiting the device solve; emptied by finish_generators
  std::vector<zd> cols;
};

struct Params {
  int M = 0, N = 0, B = 0, L = 0;
  fbst_geom_kind kind = FBST_LINE;
  int mx = 0, my = 0, bu = 0, bv = 0;
  double dx = 0, dy = 0, x0 = 0, y0 = 0;  // seconds per unit direction cosine; element offsets
  double fc = 0, omega = 0, ts = 0;
  double u0 = 0, du = 0, v0 = 0, dv = 0;
  double eps = 0, delta = 0;
  fbst_precision prec = FBST_PREC_FP32;
  unsigned flags = 0;
  int p1 = 0, p2x = 0, p2y = 0, p3 = 0;
  int p1s = 0, ls1 = 0;                   // split-output stage 1a: FFT size, first-half length
  // arbitrary positions: element coordinates (seconds per unit direction
  // cosine), oversampled grid sizes (p2x, p2y hold them too; nfy = 1 for a
  // line of beams), spreading kernel width and shape parameter
  std::vector<double> px, py;
  int nuw = 0;
  double nu_beta = 0;
  double cond_bound = 0;                  // upper bound on cond(A_b) over the beams (Sec. V)
};

// Element m's position in samples of delay per unit direction cosine.
double pos_x(const Params& p, int m);
double pos_y(const Params& p, int m);

// Validate and complete the user parameters (defaults, FFT sizes).  Returns
// FBST_OK or an error with *msg set.
fbst_status resolve_params(int M, int N, int B, const fbst_geometry* geom, const fbst_band* band,
                           const fbst_grid* grid, const fbst_options* opt, Params* out,
                           std::string* msg);

// Build every table in float64.  keep_gram_gen: also fill gram/gen.
fbst_status build_tables(const Params& p, bool keep_gram_gen, HostTables* t, std::string* msg);

// With FBST_FLAG_DEVICE_GENERATORS, build_tables leaves G1/G2 (and gen/gram)
// empty and t->cols filled; given x = A_b^{-1} e_0 [B][L] from the device
// solve, this completes them (refinement, spectra) as the host path would.
fbst_status finish_generators(const Params& p, const std::vector<zd>& x, bool keep_gram_gen,
                              HostTables* t);

// The beam grid of p (kind and B set) from fbst_grid, as fbst_plan_create
// resolves it (NULL: the eq. (thetab) grid of a line).
fbst_status resolve_grid(Params* p, const fbst_grid* grid, std::string* msg);

// For a new beam grid of a line or uniform-grid plan: t->ax (and t->ay), t->u,
// t->v and the Toeplitz first columns t->cols [B][L] of the new beams, and
// their real centred form (build_tables): A_b = D_b (R_k + delta I) D_b^H with
// D_b = diag(exp(-j 2 pi eps d s_b / L)), k = key[b] indexing the distinct
// (|u|, |v|); rcols [K][L] holds R_k + delta e_0 (as complex128, imaginary 0)
// and s [B] the centring s_b in samples.
struct SteerKeys {
  std::vector<zd> rcols;
  std::vector<int> key;
  std::vector<double> s;
};
// cols: also the complex columns t->cols (needed by a host refinement).
fbst_status build_steer_tables(const Params& p, HostTables* t, SteerKeys* k, bool cols,
                               std::string* msg);

// Beams at directions (ud, vd): K [l][d][n] = (F_u A_d^{-1})[n][l] and, when
// E is given, the projection phases E [d][m][l] = exp(j a_l tau_{d,m}); float64.
fbst_status build_direction_tables(const Params& p, const std::vector<double>& ud,
                                   const std::vector<double>& vd, std::vector<zd>* K,
                                   std::vector<zd>* E, std::string* msg);

// Off-grid beams by spline interpolation (Sec. VIII, off-grid angles) on the
// beam grid u_a = u0 + a du, v_c = v0 + c dv (beam b = a bv + c; at least
// INTERP_TAPS distinct beams along each axis that has more than one): per
// direction and axis, the first of the INTERP_TAPS consecutive grid beams
// around it and the weights of the not-a-knot cubic spline through them
// evaluated at the direction (the tensor-product spline on a plane; a line
// gets the window 0 and the weights (1, 0, ...) along v).
// first [D][2] (u, v), w [D][2][INTERP_TAPS]; float64.  frac (optional):
// [D][2], the direction's position on each axis counted in grid steps from
// the window's first beam ((u - u_first) / du; 0 along v for a line).
constexpr int INTERP_TAPS = 8;
fbst_status build_interp_table(const Params& p, const std::vector<double>& ud,
                               const std::vector<double>& vd, std::vector<int>* first,
                               std::vector<double>* w, std::string* msg,
                               std::vector<double>* frac = nullptr);

// Interpolation of beamspace vectors with the reference point at the centre
// (c_x, c_y) of the array's extent (Sec. VIII, the paper's off-grid form):
// the vector at a direction is sum_i c_i exp(j a_l (u - u_i) c_x + ...) w_i[l],
// and u - u_i = (frac - i) du.  theta [2][L] holds the per-step phases
// a_l c_x du and a_l c_y dv (radians; a_l = 2 pi f_c T_s + kappa l' per
// sample of delay, c in samples per unit direction cosine; 0 along v for a
// line).
void reference_phase_rates(const Params& p, std::vector<double>* theta);

// Beamspace nulling tables for interferer directions (uq, vq) (Sec. VIII):
// G [q L + k][b][n] = (F_b^H F_q A_q^{-1})[n][k] and, when E is given, the
// projection phases E [q][m][l] = exp(j a_l tau_{q,m}); float64.
fbst_status build_null_tables(const Params& p, const std::vector<double>& uq,
                              const std::vector<double>& vq, std::vector<zd>* G,
                              std::vector<zd>* E, std::string* msg);

// The same x by the superfast doubling Schur algorithm (superfast.h), O(L log^2 L),
// run on the host by one thread.  false if a pivot is not positive.
bool superfast_first_column(const zd* col, int L, zd* x);
// exp(-2 pi j k / PM), k < PM / 2, PM = superfast::max_fft(L): the transform
// table of the superfast solve for L coefficients.
std::vector<zd> superfast_twiddles(int L);

// Levinson recursion for a Hermitian positive definite Toeplitz matrix with
// first column col: returns x = A^{-1} e_0.  false if a pivot is not positive.
bool levinson_first_column(const zd* col, int L, zd* x);

// Real symmetric positive definite case: x = A^{-1} e_0 for A = toeplitz(col).
bool levinson_real(const double* col, int L, double* x);

// Thread-local message returned by fbst_last_error().
void set_last_error(const std::string& msg);

// In-place power-of-two DFT in float64, sign = -1 (forward) or +1 (unscaled inverse).
void fft64(zd* a, int n, int sign);

}  // namespace fbst

// Beamspace nulling tables of one plan (one device allocation):
// G_{b,q} = F_b^H F_q A_q^{-1} as [P L][B][L] (complex64), and either the
// interferer beam indices [P] (int, on-grid interferers: their rows of W are
// gathered) or the projection phases E [P][M][L] (complex64, any direction:
// their beam vectors are projected from stage 1a's output).
// With interferer vectors interpolated from the grid's (fbst_nulls_create_interp)
// neither map nor E is set and vi holds the interpolation table.
struct VectorInterp {
  const int* first = nullptr;      // [n][2]
  const double* w = nullptr;       // [n][2][INTERP_TAPS]
  const double* frac = nullptr;    // [n][2]
  const double* theta = nullptr;   // [2][L]
};

struct fbst_nulls {
  const fbst_plan* plan = nullptr;
  int P = 0;
  void* dev = nullptr;
  size_t dev_bytes = 0;
  const int* map = nullptr;
  const void* E = nullptr;
  const void* G = nullptr;
  VectorInterp vi;
};

// Beams at arbitrary directions of one plan (one device allocation):
// K_d = F_u A_d^{-1} as [L][D][N] (complex64) and either the projection
// phases E [D][M][L] (complex64; w_d projected from stage 1a's output) or,
// for fbst_directions_create_interp, the interpolation table vi (w_d
// interpolated from the grid's beamspace vectors).
struct fbst_directions {
  const fbst_plan* plan = nullptr;
  int D = 0;
  void* dev = nullptr;
  size_t dev_bytes = 0;
  const void* E = nullptr;
  const void* K = nullptr;
  VectorInterp vi;
};

// Spline-interpolated off-grid beams of one plan (device: first [D][2] ints,
// then the weights [D][2][INTERP_TAPS] as float64; host copies kept for
// queries).
struct fbst_interp {
  const fbst_plan* plan = nullptr;
  int D = 0;
  void* dev = nullptr;
  const int* first = nullptr;
  const double* w = nullptr;
  std::vector<int> host_first;
  std::vector<double> host_w;
};

// A captured and instantiated launch sequence of one plan.
struct fbst_graph {
  hipGraphExec_t exec = nullptr;
};

// The plan: parameters, optional FP64 host tables and device tables.
struct fbst_plan {
  fbst::Params p;
  bool host_only = false;
  fbst::HostTables host;           // emptied after upload unless tables are kept
  bool kept = false;
  // device memory: one allocation holding every table and the own workspace
  void* dev = nullptr;
  size_t dev_bytes = 0;
  size_t ws_bytes_per_block = 0;
  // workspace bytes per launch on top of the per-block part: the scratch of
  // the split float64 stage 2 (P3 > 8192), else 0
  size_t ws_fixed_bytes = 0;
  void* own_ws = nullptr;
  // device table pointers (element type per stage precision)
  const void* tw1 = nullptr;       // twiddles in the stage-1 type
  const void* tw2 = nullptr;       // twiddles in the stage-2 type
  const void *pre1 = nullptr, *H1 = nullptr, *post1 = nullptr, *H1a = nullptr, *H1b = nullptr;
  const void *axp = nullptr, *axH = nullptr, *axq = nullptr;
  const void *ayp = nullptr, *ayH = nullptr, *ayq = nullptr;
  const void *G1 = nullptr, *G2 = nullptr, *pre3 = nullptr, *H3 = nullptr, *post3 = nullptr;
  const void* CA = nullptr;        // FBST_FLAG_STAGE2_REFINE only
  // non-uniform stage 1b (arbitrary positions)
  const void *nu_pre = nullptr, *nu_posx = nullptr, *nu_posy = nullptr, *nu_cx = nullptr,
             *nu_cy = nullptr;
  const int* nu_order = nullptr;
  int nu_lanes = 1;
  // stage 2 in precomputed form: K [L][B][N] complex64 (own allocation), or null
  void* K = nullptr;
  size_t K_bytes = 0;
  int device = 0;
  // kernel instances: bits 0-3 stage 2 (variant bits of
  // fbst::launch_toeplitz_fu), bits 4-5 the stage-1b workgroup size (tile of
  // fbst::launch_axis_czt); chosen by fbst_autotune_ex or
  // fbst_plan_set_variant; the stage-2 instances agree to float32 rounding
  // (the persistent bit changes nothing at all), the stage-1b ones exactly
  std::atomic<int> k3_variant{0};
  double generator_ms = 0.0;       // device generator solve (FBST_FLAG_DEVICE_GENERATORS), ms
};

namespace fbst {
struct InPtrs;
struct OutPtrs;
// Whole path of nb <= MAX_LAUNCH_BLOCKS blocks (inputs xs, outputs outs) with
// the workspace [yhat | w | z] of nb blocks at ws (api.cpp).
hipError_t run_blocks(const fbst_plan* pl, int nb, const InPtrs& xs, const OutPtrs& outs, void* ws,
                      hipStream_t st);
// Whole path of nb contiguous blocks, at most chunk (<= MAX_LAUNCH_BLOCKS) per
// launch, all launches sharing the workspace of chunk blocks at ws.
hipError_t run_contiguous(const fbst_plan* pl, int nb, int chunk, const void* x, void* beams,
                          void* ws, hipStream_t st);
}  // namespace fbst
