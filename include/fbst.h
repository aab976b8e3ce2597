/*
 * fbst.h -- C ABI of the MI355X (gfx950) fast broadband beamspace
 * transformation (FBST) library, libfbst.so.
 *
 * What it computes (Singh, DeLude, Davenport, Romberg, "A Fast Broadband
 * Beamspace Transformation"): from N snapshots of an M-sensor array it forms
 * N uniform samples of each of B broadband beams (problem statement of
 * Sec. III-A).  For beam b the samples are
 *
 *     beams_b = F_u (F_b^H F_b + delta I)^{-1} F_b^H y          (eqs. betahatls, bhatls)
 *
 * with F_b the MN x L Fourier-extension matrix of eq. (FthetaH),
 * [F_b]_{(m,n),l} = exp(-j 2 pi f_c tau_{b,m}) exp(j omega_l (t_n - tau_{b,m})),
 * omega_l = 2 pi eps (l - L/2) / (L T_s), l = 1..L (eq. stfourierapprox),
 * t_n = n T_s (n = 0..N-1) and [F_u]_{n,l} = exp(j omega_l t_n).
 * The library never forms these matrices: stage 1 evaluates all F_b^H y at
 * once as two chirp-z transforms (Sec. IV, eq. DFT_1; App. B for a grid),
 * stage 2 applies (F_b^H F_b + delta I)^{-1}, a Hermitian Toeplitz inverse,
 * through its Gohberg-Semencul form by circulant-embedded FFTs, then F_u as a
 * chirp-z transform (Sec. V of the paper, "Fast Inverse").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Complex data are interleaved (re, im) pairs: complex64 = two float32,
 *   complex128 = two float64, i.e. a contiguous torch.complex64 / complex128.
 *   The I/O element type is complex128 when the plan's precision is
 *   FBST_PREC_FP64 and complex64 otherwise.
 * - x (input block) is device memory [M][N], row-major, sensor-major: sample
 *   n of element m at x[m*N + n].  For a grid, m = k*my + k2 (k indexes the x
 *   axis).  A batch of nb blocks is [nb][M][N].
 * - beams (output) is device memory [B][N]: sample n of beam b at
 *   beams[b*N + n]; for a grid b = a*bv + c (a indexes u).  A batch is
 *   [nb][B][N].  beams[b] estimates s(t_n) for a source from beam direction b,
 *   referenced to the coordinate origin of the geometry.
 * - All device pointers must be 16-byte aligned; x and beams must not alias.
 * - Asynchrony: execute calls only enqueue kernels on the given hipStream_t
 *   (NULL = the default stream) and never synchronise the host.
 * - Ownership: a plan owns its device tables (allocated in plan_create, freed
 *   in fbst_destroy).  The caller owns x, beams and any workspace.
 * - Errors: every call returns a status and never throws across the ABI;
 *   fbst_last_error() gives a thread-local message for the last failure.
 * - Thread safety: a plan is immutable after creation; executes of one plan
 *   on several streams at once are safe when each uses its own workspace.
 */
#ifndef FBST_H
#define FBST_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FBST_OK = 0,
  FBST_E_INVALID = -1,     /* an argument is null, out of range or inconsistent  */
  FBST_E_UNSUPPORTED = -2, /* valid, but outside what the library implements    */
  FBST_E_NOMEM = -3,       /* host or device allocation failed                    */
  FBST_E_DEVICE = -4       /* HIP runtime error (no device, launch or copy error) */
} fbst_status;

typedef enum { FBST_LINE = 0, FBST_GRID = 1, FBST_ARBITRARY = 2 } fbst_geom_kind;

typedef enum {
  FBST_PREC_FP32 = 0,        /* every stage in float32                                  */
  FBST_PREC_FP64_STAGE2 = 1, /* stage 1 float32; Toeplitz solve + F_u in float64          */
  FBST_PREC_FP64 = 2,        /* every stage in float64; complex128 input and output       */
  FBST_PREC_BF16_SPLIT = 3,  /* stage 1a as a blocked DFT on MFMA, bfloat16 hi/lo split   */
  FBST_PREC_FP16_SPLIT = 4   /* stage 1a as a blocked DFT on MFMA, float16 hi/lo split    */
} fbst_precision;

/* Array geometry (Sec. III: tau_{theta,m} = p_m^T theta).  Element (k, k2)
 * sits at delay coordinates px = (x0 + k) dx and py = (y0 + k2) dy, in seconds
 * per unit direction cosine, so a beam with direction cosines (u, v) has
 * delays tau = u px + v py relative to the origin (the reference point).
 * LINE: mx = M, my = 1.  GRID: mx * my = M.  dx (dy) = 0 selects
 * half-wavelength spacing at the top band edge, 1 / (2 (f_c + Omega)) (Sec. IV).
 * ARBITRARY (non-uniform array, Sec. IX, eq. DFT_non_unif): element m sits at px[m], py[m]
 * (seconds per unit direction cosine, finite; py NULL: all zero); the host
 * arrays are read during fbst_plan_create only and the plan keeps a copy;
 * mx, my, dx, dy, x0, y0 are ignored.  The spatial sum of stage 1b is then a
 * type-1 non-uniform FFT per frequency (spread onto an oversampled grid with
 * an exponential-of-semicircle kernel, FFT, deconvolve), 1-D over u for a
 * beam grid with bv = 1 and 2-D over (u, v) otherwise. */
typedef struct {
  fbst_geom_kind kind;
  int mx, my;
  double dx, dy;
  double x0, y0;
  const double* px;  /* ARBITRARY only: [M] */
  const double* py;  /* ARBITRARY only: [M] or NULL */
} fbst_geometry;

/* Band (Sec. III): carrier f_c (Hz), baseband half-bandwidth Omega (Hz) and
 * sample period T_s (s); requires 0 < T_s <= 1 / (2 Omega). */
typedef struct {
  double fc, omega, ts;
} fbst_band;

/* Beam grid, uniform in direction cosine on each axis: u_a = u0 + a du
 * (a = 0..bu-1), v_c = v0 + c dv (c = 0..bv-1).  du = 0 (dv = 0) selects the
 * grid of eq. (thetab): sin(theta) = (2b - B - 1)/(B - 1) for odd counts and
 * (2b - B - 1)/B for even counts (b = 1..B).  LINE: bu = B, bv = 1. */
typedef struct {
  int bu, bv;
  double u0, du;
  double v0, dv;
} fbst_grid;

/* Plan flags. */
#define FBST_FLAG_HOST_ONLY 1u        /* build the FP64 host tables only; no device memory,
                                         execute calls fail (introspection and CPU tests) */
#define FBST_FLAG_KEEP_HOST_TABLES 2u /* keep FP64 host copies for fbst_plan_table()      */
#define FBST_FLAG_NO_SPLIT 4u         /* stage 1a as one convolution of p1 points, even
                                         where two half-length output convolutions of
                                         p1_split points would be cheaper             */
#define FBST_FLAG_PRECOMPUTE 8u       /* stage 2 in precomputed form (the paper's FBST-
                                         Precompute variant, Sec. V / Table I): the plan
                                         builds K_b = F_u A_b^{-1} (N x L per beam) on the
                                         device with the float64 Gohberg-Semencul kernel,
                                         and execution applies it as a complex matrix
                                         product on the float32 matrix cores.  Costs
                                         8 B N L bytes of device memory (at most 16 GiB)
                                         and needs P3 <= 8192; not with FBST_PREC_FP64
                                         (otherwise FBST_E_UNSUPPORTED)                   */
#define FBST_FLAG_DEVICE_GENERATORS 32u /* solve the B Toeplitz systems for the generators
                                         x_b = A_b^{-1} e_0 (Sec. V) on the GPU during
                                         fbst_plan_create (Levinson recursion in float64,
                                         one workgroup per beam, L <= 8192), for fast
                                         plan rebuilds when the beam set changes; the
                                         columns, refinement and spectra stay on the
                                         host.  Not with FBST_FLAG_HOST_ONLY. */
#define FBST_FLAG_SUPERFAST_GENERATORS 128u /* the generators x_b = A_b^{-1} e_0 by the
                                         superfast doubling Schur algorithm (Ammar and
                                         Gragg), O(L log^2 L) per beam with FFT
                                         polynomial products in float64, instead of
                                         Levinson's O(L^2); on the host, or with
                                         FBST_FLAG_DEVICE_GENERATORS on the GPU (one
                                         workgroup per beam, L <= 4096).  Its forward
                                         error grows faster with cond(A_b) than
                                         Levinson's; the plan's refinement (cond > 1e6)
                                         applies as for Levinson                       */
#define FBST_FLAG_STAGE2_REFINE 64u /* float32 stage 2 with one step of iterative
                                         refinement (Sec. V system A_b beta = w_b):
                                         beta_1 by the Gohberg-Semencul apply, then
                                         beta = beta_1 + A_b^{-1} (w_b - A_b beta_1), the
                                         residual through the circulant embedding of A_b
                                         (its first column, a plan table of B P3 complex
                                         values).  The two Gohberg-Semencul terms can be
                                         ~100x larger than beta and cancel, which float32
                                         rounding of their FFTs turns into beam errors of a
                                         few 1e-5; the refined solve removes that.  Costs
                                         8 more P3-point transforms per beam (16 in all)
                                         and B L complex64 of workspace per block.  Only
                                         with a float32 stage 2 (FBST_PREC_FP32 and the
                                         split precisions), not with FBST_FLAG_PRECOMPUTE
                                         (otherwise FBST_E_UNSUPPORTED)                  */
#define FBST_FLAG_NU_UNFUSED 16u      /* arbitrary positions: stage 1b with the
                                         oversampled grid through device memory (spread,
                                         then one FFT pass per axis) even where a fused
                                         kernel applies (a line of beams on a grid of
                                         256..4096 points; a 2-D beam grid on 32 x 32)   */

/* Basis and solver options.  eps: band expansion epsilon > 0 (0 selects 1.01).
 * L: number of basis frequencies, even and >= 2 (0 selects 2N, i.e.
 * gamma = 2; Sec. III-A).  delta: ridge of eq. (betahatls), > 0, absolute.
 * The condition number of A_b = F_b^H F_b + delta I is about 2MN/delta (at
 * most cond_bound = 1 + M lambda_max(T)/delta, T the time Gram, reported by
 * fbst_plan_info), so float32 stage 2 needs delta of the order of the noise
 * level (e.g. sigma^2 L); the paper's delta = 1e-5 needs FBST_PREC_FP64.
 * fbst_plan_create refuses (FBST_E_UNSUPPORTED, with a message) a plan whose
 * cond_bound times the stage-2 unit roundoff (2^-24 for a float32 stage 2:
 * FBST_PREC_FP32 and the two split precisions; 2^-53 for FBST_PREC_FP64 and
 * FBST_PREC_FP64_STAGE2) exceeds 1e-2, since its beams could be off by O(1).
 * A NULL options pointer selects eps = 1.01, L = 2N, delta = 1e-5 (the
 * paper's), FBST_PREC_FP64 (complex128 input and output), flags 0. */
typedef struct {
  double eps;
  int L;
  double delta;
  fbst_precision precision;
  unsigned flags;
} fbst_options;

/* Read-only plan summary (fbst_plan_info). */
typedef struct {
  int M, N, B, L;
  int mx, my, bu, bv;
  int p1;            /* FFT size of the stage-1a (time) chirp-z               */
  int p2x, p2y;      /* FFT sizes of the stage-1b (space) chirp-z, per axis   */
  int p3;            /* FFT size of the Toeplitz apply and the F_u chirp-z      */
  fbst_precision precision;
  size_t io_elem_bytes;      /* 8 (complex64) or 16 (complex128)                */
  size_t device_bytes;       /* device tables owned by the plan                  */
  size_t workspace_per_block;/* bytes of workspace one block needs               */
  int p1_split;      /* 0, or the FFT size of stage 1a in split-output form: the
                        L outputs as two halves, each a convolution of
                        p1_split >= N + L/2 - 1 points sharing one forward FFT */
  int stage2_precomputed; /* 1 when stage 2 applies a precomputed K (FBST_FLAG_PRECOMPUTE) */
  int nu_width;      /* ARBITRARY: spreading kernel width in grid points (p2x,
                        p2y are then the oversampled grid sizes); else 0       */
  int nu_lanes;      /* ARBITRARY with bv = 1: elements spread at once per
                        frequency (1..16, chosen by the plan); else 0          */
  double cond_bound; /* upper bound on cond(F_b^H F_b + delta I) over the beams:
                        1 + M lambda_max(T) / delta, T the time Gram (Sec. V) */
  double generator_ms; /* GPU time of the last device generator solve (at plan
                          creation with FBST_FLAG_DEVICE_GENERATORS, or by
                          fbst_plan_steer; Levinson, or superfast with
                          FBST_FLAG_SUPERFAST_GENERATORS), milliseconds; else 0 */
  size_t workspace_fixed; /* workspace bytes per launch on top of
                          nblocks * workspace_per_block: the scratch of a
                          float64 stage 2 at p3 = 16384 (each transform split
                          into two halves in LDS, 128 MiB); else 0 */
} fbst_info;

typedef struct fbst_plan fbst_plan;

/* Create a plan: validates, builds every table in float64 on the host
 * (chirps, chirp-kernel spectra, the Toeplitz generator c_b(d) of Sec. V in
 * closed form, x_b = A_b^{-1} e_0 by Levinson recursion and the spectra of the
 * Gohberg-Semencul factors), uploads them in the stage precisions and
 * allocates a one-block workspace.  geometry NULL: a line of M elements,
 * lambda/2 at f_c + Omega, reference at element 0.  grid NULL: B beams on the
 * eq. (thetab) grid.  band must not be NULL.  On failure *out is NULL. */
fbst_status fbst_plan_create(int M, int N, int B, const fbst_geometry* geometry,
                             const fbst_band* band, const fbst_grid* grid,
                             const fbst_options* options, fbst_plan** out);

/* Beams of one block: x [M][N] -> beams [B][N] on hip_stream.  workspace:
 * device memory of at least fbst_workspace_bytes(plan, 1) bytes, or NULL to
 * use the plan's own one-block workspace (then calls on one plan must not
 * overlap in time).  Fails with FBST_E_INVALID on null x/beams or a
 * host-only plan. */
fbst_status fbst_execute(const fbst_plan* plan, const void* x, void* beams,
                         void* workspace, void* hip_stream);

/* Most blocks one kernel launch takes (their pointers travel in the kernel
 * arguments). */
#define FBST_MAX_LAUNCH_BLOCKS 256

/* nblocks independent blocks of one plan in one set of launches:
 * x [nblocks][M][N] -> beams [nblocks][B][N], processed chunk blocks per
 * launch, chunk = min(nblocks, max_chunk, FBST_MAX_LAUNCH_BLOCKS)
 * (max_chunk <= 0: no limit of its own).  workspace: at least
 * fbst_workspace_bytes(plan, chunk) bytes, or NULL when chunk == 1. */
fbst_status fbst_execute_batched(const fbst_plan* plan, int nblocks, int max_chunk,
                                 const void* x, void* beams, void* workspace,
                                 void* hip_stream);

/* Streaming over one recording (Sec. III, streaming remark: contiguous and
 * possibly overlapping batches of snapshots): x [M][T] (row-major, T samples
 * per sensor, the plan's I/O type) is cut into windows of N samples starting
 * every hop samples (hop < N overlaps them), nblocks = (T - N) / hop + 1, and
 * beams [nblocks][B][N] receives the beams of each window (time origin at the
 * window's first sample).  Launches as fbst_execute_batched (chunk =
 * min(nblocks, max_chunk, FBST_MAX_LAUNCH_BLOCKS); workspace of
 * fbst_workspace_bytes(plan, chunk) bytes, or NULL when chunk == 1).  Stage 1a
 * reads the windows in place (no copy).  T >= N and hop >= 1, else
 * FBST_E_INVALID. */
fbst_status fbst_execute_stream(const fbst_plan* plan, long long T, int hop, const void* x,
                                void* beams, void* workspace, int max_chunk, void* hip_stream);

/* One stage, for per-stage parity and timing.  Element types are the plan's
 * stage types (complex64, or complex128 for FBST_PREC_FP64; stage 2 input is
 * the stage-1 type).
 *   stage 0 (time chirp-z, Sec. IV):   in x [nb][M][N]  -> out Yhat [nb][M][L],
 *            Yhat[m][l-1] = sum_n x[m][n] exp(-j omega_l t_n);
 *   stage 1 (space chirp-z, eq. DFT_1 / App. B): in Yhat -> out W [nb][B][L],
 *            W[b][l-1] = [F_b^H x]_l; a grid or an arbitrary array needs
 *            workspace of fbst_workspace_bytes(plan, nb) bytes (else may be NULL);
 *   stage 2 (Sec. V):                  in W -> out beams [nb][B][N]; a plan
 *            with FBST_FLAG_STAGE2_REFINE needs workspace of
 *            fbst_workspace_bytes(plan, nb) bytes (may be NULL when nb == 1);
 *            a float64 stage 2 at p3 = 16384 uses workspace_fixed bytes of
 *            it as scratch (NULL: the plan's own, any nb). */
fbst_status fbst_execute_stage(const fbst_plan* plan, int stage, int nblocks,
                               const void* in, void* out, void* workspace,
                               void* hip_stream);

/* ---- Graph capture and tuning of batched launches ---------------------- */
typedef struct fbst_graph fbst_graph;

/* Capture the launches of fbst_execute_batched(plan, nblocks, max_chunk, x,
 * beams, workspace) into an instantiated HIP graph bound to these buffers
 * (they must stay valid while the graph is used).  The capture runs on a
 * private stream and executes nothing.  The graph holds no memset node. */
fbst_status fbst_graph_create(const fbst_plan* plan, int nblocks, int max_chunk, const void* x,
                              void* beams, void* workspace, fbst_graph** out);

/* Replay the captured launches on hip_stream (asynchronous). */
fbst_status fbst_graph_launch(const fbst_graph* graph, void* hip_stream);

/* Free a graph (after its launches finished); NULL is a no-op. */
void fbst_graph_destroy(fbst_graph* graph);

/* Autotune the blocks per launch of fbst_execute_batched for nblocks blocks of
 * this plan: times chunk = 1, 2, 4, ... (<= min(nblocks, FBST_MAX_LAUNCH_BLOCKS)) on the given
 * buffers (x [nblocks][M][N], beams, workspace of fbst_workspace_bytes(plan,
 * min(nblocks, FBST_MAX_LAUNCH_BLOCKS)) bytes) on hip_stream, synchronising it, and returns the
 * fastest chunk and its ms per batch.  Results are cached per plan shape and
 * precision for the process; force != 0 re-measures.  beams is overwritten. */
fbst_status fbst_autotune(const fbst_plan* plan, int nblocks, const void* x, void* beams,
                          void* workspace, void* hip_stream, int force, int* best_chunk,
                          float* best_ms);

/* Compiled instances of the stage-2 kernel a plan can launch (variant bits).
 * FBST_VARIANT_K3_PERSISTENT leaves the beams bit-identical;
 * FBST_VARIANT_K3_SINGLE changes them at the level of float32 rounding (the
 * two branches' products are combined in another rounding order):
 *   FBST_VARIANT_K3_SINGLE      the two Gohberg-Semencul branches in sequence in
 *                               one LDS buffer, instead of as one dual transform
 *                               in two buffers;
 *   FBST_VARIANT_K3_PERSISTENT  a persistent grid: as many workgroups as are
 *                               resident at once, each working through a
 *                               contiguous range of (block, beam) rows, instead
 *                               of one workgroup per row group.
 * Variants 1, 2, 3 and 5 exist for a float32 stage 2 (FBST_PREC_FP32 and the
 * split precisions) at P3 >= 1024, without FBST_FLAG_PRECOMPUTE or
 * FBST_FLAG_STAGE2_REFINE; such plans start with FBST_VARIANT_K3_SINGLE, the
 * others with 0. */
#define FBST_VARIANT_K3_SINGLE 1
#define FBST_VARIANT_K3_PERSISTENT 2
#define FBST_VARIANT_K3_WAVES3 4   /* with FBST_VARIANT_K3_SINGLE only: registers
                                      allocated for 3 waves per SIMD (spills)    */
/* Stage-1b instances (bits 4-5, combined with any stage-2 variant): the
 * space chirp-z's workgroup holds half (FBST_VARIANT_K2_TILE_HALF) or twice
 * (FBST_VARIANT_K2_TILE_DOUBLE) the default number of frequencies; beams are
 * bit-identical.  For lines and uniform grids with a float32 stage 1. */
#define FBST_VARIANT_K2_TILE_HALF 16
#define FBST_VARIANT_K2_TILE_DOUBLE 32

/* As fbst_autotune, also over the stage-2 variants this plan can launch
 * (chunk x variant), and leaves the fastest variant set on the plan (the only
 * state a plan changes after creation; results stay within float32 rounding
 * of the untuned plan's).  The
 * cache key is (device architecture, M, N, B, L, geometry and beam-grid
 * shape, precision, flags, nblocks).  best_variant may be NULL. */
fbst_status fbst_autotune_ex(const fbst_plan* plan, int nblocks, const void* x, void* beams,
                             void* workspace, void* hip_stream, int force, int* best_chunk,
                             int* best_variant, float* best_ms);

/* Select the stage-2 variant (FBST_E_UNSUPPORTED when it is not compiled
 * for this plan); takes effect for launches issued afterwards.  Not to be
 * called while another thread issues launches of the plan. */
fbst_status fbst_plan_set_variant(const fbst_plan* plan, int variant);

/* The plan's stage-2 variant (-1 on a NULL plan). */
int fbst_plan_variant(const fbst_plan* plan);

/* ---- Beamspace interference nulling (Sec. VIII, eq. interfer_beam_space) -- */
typedef struct fbst_nulls fbst_nulls;

/* Interferers at the plan's own beams beams[0..n_interferers-1] (1..64
 * indices in [0, B)).  Builds, in float64 on the host, G_{b,q} =
 * F_b^H F_q (F_q^H F_q + delta I)^{-1} for every beam b and interferer q
 * (closed-form cross-Gram, Gohberg-Semencul applies of the refined
 * generator of A_q; about 3e4 B P L^2 log2(L) flops on the host) and uploads
 * it as complex64: 8 B P L^2 bytes of device memory (at most 16 GiB, else
 * FBST_E_UNSUPPORTED).  Several interferers are removed as the sum of their
 * separate projections, as in the paper.  Not for FBST_PREC_FP64 plans
 * (FBST_E_UNSUPPORTED).  The plan must outlive it. */
fbst_status fbst_nulls_create(const fbst_plan* plan, int n_interferers, const int* beams,
                              fbst_nulls** out);

/* Interferers at arbitrary directions (u[i], v[i]) (direction cosines; v
 * NULL or ignored for a line), on or off the beam grid (Sec. VIII: the
 * interferer need not align with the grid).  As fbst_nulls_create, plus the
 * projection phases exp(j (2 pi f_c + omega_l) tau_{q,m}) (8 P M L bytes):
 * each interferer's beam vector w_q = F_q^H y is formed exactly from stage
 * 1a's output (M L complex products per interferer and block) instead of
 * being interpolated from neighbouring grid beams. */
fbst_status fbst_nulls_create_directions(const fbst_plan* plan, int n_interferers, const double* u,
                                         const double* v, fbst_nulls** out);

/* Interferers at arbitrary directions (u[i], v[i]) within the beam grid,
 * with each interferer's beam vector w_q estimated the paper's way (Sec. VIII,
 * closing paragraph of interference cancellation: off-grid beam vectors are
 * interpolated from the surrounding grid beam vectors): stage 1 forms W for
 * the grid, and w_q is the not-a-knot cubic spline in direction cosine
 * through the 8 (8 x 8 on a planar grid) grid vectors around the interferer,
 * taken with their reference point moved to the centre of the array's extent
 * (the vectors vary more slowly with direction that way; the result is
 * referred back to the origin).  G_{b,q} as in fbst_nulls_create_directions,
 * at the interferer's own direction; no projection phases are stored.
 * Needs at least 8 distinct grid beams along each axis with more than one
 * (FBST_E_UNSUPPORTED) and directions inside the grid (FBST_E_INVALID; no
 * extrapolation); v required for a planar grid.  Executes with
 * fbst_execute_nulled and fbst_workspace_bytes_nulled. */
fbst_status fbst_nulls_create_interp(const fbst_plan* plan, int n_interferers, const double* u,
                                     const double* v, fbst_nulls** out);

/* Free nulling tables (after their launches finished); NULL is a no-op. */
void fbst_nulls_destroy(fbst_nulls* nulls);

/* Workspace bytes of fbst_execute_nulled for nblocks blocks per launch
 * (0 on NULL arguments). */
size_t fbst_workspace_bytes_nulled(const fbst_plan* plan, const fbst_nulls* nulls, int nblocks);

/* Beams with the interferers nulled: as fbst_execute_batched (x [nblocks][M][N]
 * complex64 -> beams [nblocks][B][N]), with, between the two stages,
 *   w~_b = w_b - sum_q G_{b,q} w_q
 * on the float32 matrix cores, and stage 2 applied to w~.  workspace (required)
 * holds fbst_workspace_bytes_nulled(plan, nulls, chunk) bytes. */
fbst_status fbst_execute_nulled(const fbst_plan* plan, const fbst_nulls* nulls, int nblocks,
                                int max_chunk, const void* x, void* beams, void* workspace,
                                void* hip_stream);

/* ---- Beams at arbitrary directions (Sec. VIII, off-grid angles) ----------- */
typedef struct fbst_directions fbst_directions;

/* Beams at directions (u[i], v[i]) (direction cosines; v NULL or ignored for a
 * line), on or off the plan's grid.  Builds in float64 on the host, per
 * direction d, K_d = F_u (F_d^H F_d + delta I)^{-1} (N x L, Gohberg-Semencul
 * applies of the refined generator) and the projection phases of F_d^H, and
 * uploads them as complex64: 8 D L (N + M) bytes (at most 16 GiB).  The
 * paper interpolates the beam vector of an off-grid direction from
 * neighbouring grid beam vectors with a spline (fbst_directions_create_interp);
 * here it is projected exactly, so the beam is the regularised least-squares
 * beam of that direction, at a cost of M L + N L complex products per
 * direction and block.  Not for FBST_PREC_FP64 plans (FBST_E_UNSUPPORTED).  The plan must
 * outlive it. */
fbst_status fbst_directions_create(const fbst_plan* plan, int n_directions, const double* u,
                                   const double* v, fbst_directions** out);

/* The paper's off-grid beams (Sec. VIII, off-grid angle interpolation): for
 * each direction d, w_d is estimated from the beamspace vectors of the grid
 * beams around it and the beam is formed from it like a grid beam,
 *     b_d = K_d w_d,  K_d = F_u (F_d^H F_d + delta I)^{-1},
 * with the direction's own Toeplitz system.  w_d is the not-a-knot cubic
 * spline in direction cosine through the 8 grid vectors j-3 .. j+4 around the
 * direction (window shifted inward at the ends; 8 x 8 with the tensor-product
 * spline on a planar grid), interpolated with the reference point moved to
 * the centre of the array's extent and referred back to the origin:
 *     w_d[l] = sum_i c_i exp(j a_l (u_d - u_i) c_x) w_i[l]   (and along v),
 * a_l = 2 pi f_c + omega_l.  K_d as in fbst_directions_create; no projection
 * phases: 8 D L N bytes plus 160 bytes per direction and 16 L bytes.  Needs
 * at least 8 distinct grid beams along each axis with more than one
 * (FBST_E_UNSUPPORTED) and directions inside the grid (FBST_E_INVALID; no
 * extrapolation); v required for a planar grid.  Executes with
 * fbst_execute_directions: stage 1 for the whole grid, the interpolation,
 * then the K_d product; its workspace (fbst_workspace_bytes_directions)
 * holds the path's own per-block workspace plus D L complex64 per block. */
fbst_status fbst_directions_create_interp(const fbst_plan* plan, int n_directions,
                                          const double* u, const double* v,
                                          fbst_directions** out);

/* Free direction tables (after their launches finished); NULL is a no-op. */
void fbst_directions_destroy(fbst_directions* dirs);

/* Workspace bytes of fbst_execute_directions for nblocks blocks per launch. */
size_t fbst_workspace_bytes_directions(const fbst_plan* plan, const fbst_directions* dirs,
                                       int nblocks);

/* x [nblocks][M][N] complex64 -> beams [nblocks][D][N] at the directions:
 * stage 1a, w_d[l] = sum_m Yhat[m][l] exp(j (2 pi f_c + omega_l) tau_{d,m}),
 * and b_d = K_d w_d on the float32 matrix cores, chunk = min(nblocks,
 * max_chunk, FBST_MAX_LAUNCH_BLOCKS) blocks per launch; workspace required. */
fbst_status fbst_execute_directions(const fbst_plan* plan, const fbst_directions* dirs,
                                    int nblocks, int max_chunk, const void* x, void* beams,
                                    void* workspace, void* hip_stream);

/* ---- Off-grid beams by spline interpolation (Sec. VIII, off-grid angles) --- */
typedef struct fbst_interp fbst_interp;

/* The paper's interpolated off-grid beam: for each direction (u[d], v[d])
 * (direction cosines) and each axis of the beam grid u_a = u0 + a du,
 * v_c = v0 + c dv (beam b = a bv + c), the 8 consecutive grid beams
 * j-3 .. j+4 with x_j <= x < x_{j+1} (the window shifted inward at the ends of
 * the axis) and the real weights of the cubic spline with not-a-knot ends
 * through them, evaluated at the direction (computed in float64 on the host,
 * kept there and uploaded: 136 bytes per direction).  A line of beams
 * (bv == 1, v NULL or ignored) interpolates 8 beams along u; a planar grid
 * (bv > 1, v required) takes the tensor-product spline over 8 x 8 beams.
 * Each axis with more than one beam needs at least 8 distinct beams
 * (FBST_E_UNSUPPORTED otherwise); directions must lie within the grid
 * (FBST_E_INVALID otherwise: no extrapolation).  1..65536 directions.  For a
 * plan created with FBST_FLAG_HOST_ONLY only the host table is built
 * (fbst_interp_table works, fbst_execute_interp returns FBST_E_INVALID).  The
 * plan must outlive it. */
fbst_status fbst_interp_create(const fbst_plan* plan, int n_directions, const double* u,
                               const double* v, fbst_interp** out);

/* Free interpolation tables (after their launches finished); NULL is a no-op. */
void fbst_interp_destroy(fbst_interp* interp);

/* Host copy of the table: first [D][2] (first grid index of the u and the v
 * window; v is 0 for a line) and w [D][2][8] (float64 weights along u, then
 * along v; a line has (1, 0, ..., 0) along v); either may be NULL.
 * FBST_E_INVALID on NULL interp. */
fbst_status fbst_interp_table(const fbst_interp* interp, int* first, double* w);

/* beams [nblocks][B][N] (device; complex64, complex128 for FBST_PREC_FP64
 * plans; the output of fbst_execute*) -> out [nblocks][D][N] (device, same
 * type): out[blk][d][n] = sum_{i,j} wu[d][i] wv[d][j]
 * beams[blk][(a0 + i) bv + c0 + j][n] with (a0, c0) = first[d], one launch on
 * hip_stream, no workspace.  nblocks == 0 is a no-op. */
fbst_status fbst_execute_interp(const fbst_interp* interp, int nblocks, const void* beams,
                                void* out, void* hip_stream);

/* ---- Allocation-free execution ------------------------------------------
 * For callers that cannot allocate device memory while they run: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * fbst_execute_static is fbst_execute_batched with its workspace taken from
 * a fixed device array inside libfbst.so (FBST_STATIC_SCRATCH_BYTES per GPU,
 * held by every GPU the library runs on until the process ends) instead of
 * caller or plan memory: it calls no allocating routine.  Blocks are
 * processed min(nblocks, FBST_MAX_LAUNCH_BLOCKS, scratch / workspace per
 * block) per launch.  The plan's device must be the current device.  Every
 * call on a GPU shares that GPU's array, so calls that overlap in time on one
 * GPU (on different streams or threads) race and must be serialised by the
 * caller; the array's contents from earlier calls are never read.  Errors:
 * FBST_E_INVALID on a NULL plan, x or beams, a host-only plan or another
 * current device; FBST_E_UNSUPPORTED when one block's workspace
 * (fbst_workspace_bytes(plan, 1)) exceeds the array (so every float64 stage
 * 2 at p3 = 16384, whose fixed scratch alone is 128 MiB).  nblocks == 0 is a
 * no-op.  Layouts as fbst_execute_batched.
 * ------------------------------------------------------------------------ */
#define FBST_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
fbst_status fbst_execute_static(const fbst_plan* plan, int nblocks, const void* x, void* beams,
                                void* hip_stream);

/* Size of that array in bytes (FBST_STATIC_SCRATCH_BYTES). */
size_t fbst_static_scratch_bytes(void);

/* Point an existing plan at a new beam grid (same bu and bv; u0, du, v0,
 * dv as in fbst_plan_create, du = 0 for the eq. (thetab) grid), for beam
 * sets that change while the array streams (Sec. V: the generators of the
 * new beams computed on the fly).  For a line or uniform grid: the host
 * builds the new stage-1b chirps and the Toeplitz first columns in closed
 * form; the GPU solves the new generators (Levinson, or the superfast
 * doubling Schur algorithm with FBST_FLAG_SUPERFAST_GENERATORS) and forms
 * the Gohberg-Semencul spectra in place of the old (with refinement on the
 * host when 2MN/delta > 1e6, as at plan creation).  Synchronises hip_stream
 * first (launches already issued on it finish with the old beams) and
 * returns when the new tables are in place; the plan must not be in use on
 * other streams meanwhile.  fbst_info.generator_ms reports the GPU solve.
 * Tables made from the plan earlier (nulls, directions, interpolation)
 * keep the old grid: recreate them.  Errors: FBST_E_INVALID (NULL plan,
 * host-only plan, another current device, a grid that changes bu or bv, a
 * system not positive definite: the plan is then unchanged);
 * FBST_E_UNSUPPORTED for arbitrary arrays, FBST_FLAG_PRECOMPUTE and
 * FBST_FLAG_STAGE2_REFINE plans. */
fbst_status fbst_plan_steer(fbst_plan* plan, const fbst_grid* grid, void* hip_stream);

/* Workspace bytes for nblocks blocks processed in one launch (0 on NULL plan):
 * nblocks * workspace_per_block + workspace_fixed (fbst_info). */
size_t fbst_workspace_bytes(const fbst_plan* plan, int nblocks);

/* Device bytes owned by the plan (tables + its one-block workspace). */
size_t fbst_plan_device_bytes(const fbst_plan* plan);

/* Fill *info; FBST_E_INVALID on NULL arguments. */
fbst_status fbst_plan_info(const fbst_plan* plan, fbst_info* info);

/* FP64 host tables kept by plans created with FBST_FLAG_HOST_ONLY or
 * FBST_FLAG_KEEP_HOST_TABLES, copied to host memory dst (bytes available):
 *   FBST_TABLE_BEAM_U, FBST_TABLE_BEAM_V: double [B], direction cosines;
 *   FBST_TABLE_GRAM:      complex128 [B][L], first column of A_b = F_b^H F_b
 *                         + delta I, i.e. c_b(d) + delta [d == 0];
 *   FBST_TABLE_GENERATOR: complex128 [B][L], x_b = A_b^{-1} e_0.
 * FBST_E_INVALID if the table is absent or bytes is too small. */
#define FBST_TABLE_BEAM_U 0
#define FBST_TABLE_BEAM_V 1
#define FBST_TABLE_GRAM 2
#define FBST_TABLE_GENERATOR 3
fbst_status fbst_plan_table(const fbst_plan* plan, int table, void* dst, size_t bytes);

/* Free the plan and its device tables (after work using it has finished).
 * NULL is a no-op. */
void fbst_destroy(fbst_plan* plan);

/* Thread-local text of the last failure ("" if none). */
const char* fbst_last_error(void);

/* Library version string. */
const char* fbst_version(void);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of independent blocks of many resident plans.
 *
 * The method's blocks are independent (Sec. III-A streaming remark; Sec. VI
 * notes the per-beam and per-frequency independence), so a server can batch
 * whatever blocks are waiting.  A server owns a device workspace budget, a
 * few launch streams and one scheduler thread.  Whenever a stream is idle
 * the scheduler takes the oldest waiting request, gathers up to max_batch
 * waiting requests of the same plan (arrival order), admits them when their
 * workspace fits in the budget (halving the batch until it does) and launches
 * the whole path for them with per-block input/output pointers.  Launches on
 * different streams overlap on the GPU; requests arriving meanwhile join the
 * next launch.  Each block's result is bitwise the same alone or batched.
 * Streams are created with default priority.
 * ------------------------------------------------------------------------ */
typedef struct fbst_server fbst_server;

typedef struct {
  size_t workspace_bytes; /* device workspace for blocks in flight (> 0)            */
  int streams;            /* concurrent launch streams, 1..16                        */
  int max_batch;          /* blocks of one plan per launch, 1..FBST_MAX_LAUNCH_BLOCKS */
  int device;             /* HIP device, or -1 for the calling thread's current one  */
} fbst_server_options;

typedef struct {
  unsigned long long tag; /* the caller's tag of the request                         */
  int status;             /* FBST_OK; FBST_E_NOMEM if the budget cannot hold one block
                             of its plan; FBST_E_DEVICE on a launch or device error;
                             FBST_E_INVALID if cancelled by fbst_server_destroy       */
  int batch;              /* blocks in the launch that served it                     */
  double submit_us;       /* server clock (fbst_server_clock_us) at submit           */
  double start_us;        /* ... when its launch was issued                           */
  double done_us;         /* ... when the scheduler saw the launch complete            */
} fbst_completion;

/* Create a server (NULL options: 1 GiB workspace, 4 streams, batches of 16,
 * current device).  Allocates the workspace and starts the scheduler. */
fbst_status fbst_server_create(const fbst_server_options* options, fbst_server** out);

/* Queue one block: x [M][N] -> beams [B][N] of plan (layouts as fbst_execute).
 * Returns at once; x and beams must stay valid, and beams untouched, until the
 * request's completion has been polled.  The plan must outlive its requests.
 * x must already hold its data when this is called: the server's streams do
 * not wait on the caller's streams, so device work that writes x (on any
 * stream) must have completed (e.g. hipStreamSynchronize of the producing
 * stream) before the submit. */
fbst_status fbst_server_submit(fbst_server* server, const fbst_plan* plan, const void* x,
                               void* beams, unsigned long long tag);

/* Move up to max completions (oldest first) into out; returns how many, or a
 * negative status on invalid arguments. */
int fbst_server_poll(fbst_server* server, fbst_completion* out, int max);

/* Block until nothing is queued or running (timeout_s <= 0: no timeout);
 * FBST_E_DEVICE on timeout. */
fbst_status fbst_server_drain(fbst_server* server, double timeout_s);

/* The server's clock in microseconds since creation (steady clock). */
double fbst_server_clock_us(const fbst_server* server);

/* Stop the scheduler: queued requests are completed as cancelled, running
 * launches are waited for, then the streams and workspace are freed.
 * NULL is a no-op. */
void fbst_server_destroy(fbst_server* server);

#ifdef __cplusplus
}
#endif

#endif /* FBST_H */
