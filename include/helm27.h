/*
 * helm27 -- wavelength-adaptive 27-point frequency-domain Helmholtz operator
 * and solver for AMD Instinct MI355X (gfx950).
 *
 * The method (Aghamiry, Gholami, Combe, Operto, "Accurate 3D frequency-domain
 * seismic wave modeling with the wavelength-adaptive 27-point finite-difference
 * stencil"):
 *   - a table of stencil weights over G (grid points per wavelength), each
 *     entry minimising numerical dispersion for its G, smoothed along G by a
 *     Tikhonov term (Sec. 2.2);
 *   - an impedance matrix [M + S] whose every row uses the weights of its local
 *     G = c / (f h) (Sec. 3.1, "GA"), with a 27-point weighted stiffness
 *     (Sec. 2.1, weighted sum over the Cartesian, 45-degree-rotated and
 *     cube-diagonal stencils), a consistent mass (Sec. 2.1, second form:
 *     bulk modulus at the collocation point) and PML by complex coordinate
 *     stretching (Sec. 2.1);
 *   - solutions for point sources (Sec. 3.1).  The paper factorises the matrix
 *     with a sparse direct solver; this library solves it matrix-free with
 *     restarted GMRES preconditioned by a complex-shifted-Laplacian multigrid
 *     whose smoother is the same stencil kernel, with FP64 iterative refinement
 *     around complex-FP32 inner iterations.
 *
 * Conventions
 *   - Grid order: x fastest, lin = i + nx * (j + ny * k).  A multi-vector of
 *     nrhs right-hand sides is [nrhs][nz][ny][nx], contiguous.
 *   - Complex data are interleaved (re, im): HELM27_C64 = 2 x float,
 *     HELM27_C128 = 2 x double.
 *   - Time convention exp(-i omega t); outgoing waves decay in the PML.
 *   - Every call returns an int status: HELM27_OK (0) or a negative code
 *     below; helm27_strerror() names it.  No exception crosses this boundary.
 *   - Ownership: the caller owns every buffer it passes (host or device
 *     pointers as stated per argument); the library owns everything behind
 *     its handles and frees it in the matching *_destroy call.
 *   - Threading: a context and the objects made from it may be used by one
 *     host thread at a time; the serving calls are internally synchronised.
 *   - Streams: a NULL stream means the default (null) stream of the device.
 */
#ifndef HELM27_H
#define HELM27_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define HELM27_OK         0
#define HELM27_EINVAL    -1   /* bad argument (null pointer, bad size, bad flag) */
#define HELM27_ENOMEM    -2   /* device or host allocation failed */
#define HELM27_EADMIT    -3   /* request larger than the context's HBM budget */
#define HELM27_ENOCONV   -4   /* iteration limit reached before the tolerance */
#define HELM27_ENUMERIC  -5   /* NaN / Inf in the data or a Krylov breakdown */
#define HELM27_EDEVICE   -6   /* a HIP call failed */
#define HELM27_ERANGE    -7   /* a source outside the grid or inside the PML */
#define HELM27_ENOTFOUND -8   /* unknown serving ticket */
#define HELM27_EAGAIN    -9   /* serving result not ready yet */

/* ---- dtypes, variants, flags -------------------------------------------- */
#define HELM27_C64   1        /* complex float  (2 x fp32) */
#define HELM27_C128  2        /* complex double (2 x fp64) */

#define HELM27_RECOMPUTE 0    /* apply: coefficients rebuilt from table index + velocity */
#define HELM27_STORED    1    /* apply: 27 stored complex coefficients per point */
#define HELM27_STORED_T  2    /* apply the transpose A^T from the stored coefficients (adjoint
                                 problems of waveform inversion, Sec. 1; A^H u = conj(A^T conj(u))) */

/* assembly flags (helm27_assemble) */
#define HELM27_WEIGHTS_GA     0x0   /* per-row table entry of the row's own G (Sec. 3.1 "GA") */
#define HELM27_WEIGHTS_FIXED  0x1   /* table entry 0 on every row ("G4" / "Gm", Sec. 3.1) */
#define HELM27_WEIGHTS_GAM    0x2   /* mean of the 27 stencil points' entries (Sec. 3.1 "GAm") */
#define HELM27_STORE_C64      0x10  /* also keep 27 stored complex-float coefficients per point */
#define HELM27_STORE_C128     0x20  /* also keep 27 stored complex-double coefficients per point */
#define HELM27_MASS_A         0x80  /* first consistent-mass form (Sec. 2.1, eq. 8): the mass term of row i
                                       takes each neighbour's own bulk modulus, A = S + M diag(k^2),
                                       instead of the collocation point's (second form, the default) */
#define HELM27_EXTEND_TABLE   0x40  /* widen the table (same axis, step and fit settings) until no row
                                       clamps (see helm27_solve_opts.mg_coarse_table for the coarse
                                       multigrid levels) */

/* ---- opaque handles ----------------------------------------------------- */
typedef struct helm27_ctx   helm27_ctx;
typedef struct helm27_table helm27_table;
typedef struct helm27_op    helm27_op;

/* Create a context on HIP device `device`.  `hbm_budget_bytes` bounds the
 * device memory that serving admits at once (0 = 90% of the free memory).
 * Errors: EINVAL (bad device), EDEVICE. */
int  helm27_create(helm27_ctx** out, int device, size_t hbm_budget_bytes);
void helm27_destroy(helm27_ctx* ctx);
const char* helm27_strerror(int status);

/* ---- (a0) weight table ---------------------------------------------------
 * Options of the dispersion fit (Sec. 2.2).  NULL selects the defaults:
 * theta and phi both on 0, 10, 20, 30, 40 degrees; first-difference smoother;
 * a G-uniform axis. */
#define HELM27_SPACING_G     0   /* abscissae G_i = g_min + i dg */
#define HELM27_SPACING_INVG  1   /* abscissae s_i = g_min + i dg with s = 1/G (the paper's
                                    axis, figure caption of the dispersion curves:
                                    1/G from 0 to 0.4 by 0.001) */
typedef struct {
    int    n_angles;        /* angles per axis (default 5) */
    double angle_step_deg;  /* spacing (default 10) */
    int    diff_order;      /* 1 = first difference (default), 2 = second */
    int    spacing;         /* HELM27_SPACING_G (default) or HELM27_SPACING_INVG */
} helm27_table_opts;

/* Build the adaptive table on the host in FP64 (Sec. 2.2): for
 * G_i = g_min + i dg (i = 0 .. round((g_max - g_min)/dg)) -- or, with
 * HELM27_SPACING_INVG, for s_i = 1/G_i = g_min + i dg, where g_min, g_max and
 * dg bound and step s and g_min may be 0 (G infinite; every dispersion row
 * vanishes there and the smoothing term alone fixes the entry) -- solve
 *     min ||H w - g||^2 + lambda ||D P w||^2
 * over the five free weights of every G_i by banded Givens QR of the stacked
 * matrix [H; sqrt(lambda) D P] (unknowns in G-major order, so the stacked
 * matrix has bandwidth 10).  The rows of H are the v~ = 1 equations of the
 * dispersion analysis with w_s3 and the last mass weight eliminated (H_2
 * including its constant 1/2, as the elimination gives).
 * lambda = 0 decouples the G values; each is then solved for its minimum-norm
 * least-squares weights (one-sided Jacobi SVD), since alone it is rank deficient.
 * Errors: EINVAL (g_min <= 0 on the G axis or < 0 on the 1/G axis, dg <= 0,
 * g_max < g_min, lambda < 0, lambda = 0 on the 1/G axis, more than 65535
 * entries, bad options), ENUMERIC, ENOMEM. */
int helm27_build_table(helm27_ctx* ctx, double g_min, double g_max, double dg, double lambda,
                       const helm27_table_opts* opts, helm27_table** out);

/* A table from caller-given weights on the axis `spacing` (abscissae
 * g_min + i dg of G, or of s = 1/G): `w5` is host memory [n_g][5] holding
 * (w_s1, w_s2, w_m0, w_m1, w_m2) per entry, the rest following from
 * sum w_s = 1 and w_m0 + 6 w_m1 + 12 w_m2 + 8 w_m3 = 1.  n_g = 1 gives fixed
 * weights.  The data are copied.  Such a table cannot be widened by
 * HELM27_EXTEND_TABLE (its fit settings are unknown).  Errors: EINVAL. */
int helm27_table_from_weights(helm27_ctx* ctx, int spacing, double g_min, double dg, int n_g,
                              const double* w5, helm27_table** out);

/* Non-adaptive weights (Sec. 2.2, joint misfit over several G with one weight
 * vector, e.g. G = 4 for "G4" and G = 4, 6, 8, 10 for "Gm"), computed by
 * one-sided Jacobi SVD in FP64 on the host.  A single G gives a rank-3
 * system whose least-squares solutions form a plane: w5_near (host [5], the
 * free weights w_s1, w_s2, w_m0, w_m1, w_m2, or NULL) picks the one closest
 * to it, NULL the minimum-norm one.  For G = 4 the minimum-norm stencil has
 * spurious modes (its stiffness symbol changes sign at q h = (pi, pi, 0) and
 * its mass symbol goes negative) and preconditioned iterative solves of it
 * do not converge; the smoothed table's entry at G = 4 as w5_near gives a
 * stencil with the same phase velocities at G = 4 and positive symbols.
 * Returns a one-entry table to be assembled with HELM27_WEIGHTS_FIXED.
 * g_list: host [n_list].  Errors: EINVAL, ENUMERIC, ENOMEM. */
int helm27_fit_fixed(helm27_ctx* ctx, const double* g_list, int n_list, const helm27_table_opts* opts,
                     const double* w5_near, helm27_table** out);

/* Copy the table out: w7 (host, caller-owned, [n_g][7] or NULL) receives
 * (w_s1, w_s2, w_s3, w_m0, w_m1, w_m2, w_m3) per entry (per-point mass
 * weights); n_g, g_min, dg may be NULL.  Errors: EINVAL. */
int helm27_table_weights(const helm27_table* t, double* w7, int* n_g, double* g_min, double* dg);
/* The table's axis: spacing (HELM27_SPACING_*), first abscissa, step, entries
 * (any pointer may be NULL).  Errors: EINVAL. */
int helm27_table_axis(const helm27_table* t, int* spacing, double* v_min, double* dv, int* n_g);
void helm27_table_destroy(helm27_table* t);

/* ---- (a1) assembly ------------------------------------------------------- */
typedef struct {
    int    npml[3];   /* PML layer width in nodes along x, y, z (both faces); 0 = none */
    double R;         /* theoretical reflection coefficient (default 1e-3 if <= 0) */
    double c_ref;     /* velocity used for the damping strength; <= 0: max of the model */
} helm27_pml;

typedef struct {
    int      nx, ny, nz;
    double   h, freq, omega;
    int      n_g;
    int64_t  n_clamped;     /* points whose G fell outside the table (clamped) */
    double   g_min_model;   /* smallest / largest G = c/(f h) of the model */
    double   g_max_model;
    size_t   device_bytes;  /* device memory held by the operator */
    /* recompute-kernel shape (helm27_set_* / helm27_tune); auto_tile = 1 while
     * every launch still chooses its own shape from its work size */
    int      auto_tile, kernel_variant, rows_fp32, rows_fp64, zchunk, rhs_block, rhs_order;
    /* the table the operator uses (the given one, or its widened copy under
     * HELM27_EXTEND_TABLE): axis, first abscissa, step (n_g entries above) */
    int      table_spacing;
    double   table_min, table_step;
} helm27_op_desc;

/* Build the operator for velocity `vel` (float32 [nz][ny][nx], host or device
 * pointer, copied), grid step h (m), frequency freq (Hz), PML `pml` (NULL: 8
 * nodes, R = 1e-3) and `flags` (HELM27_WEIGHTS_*, HELM27_STORE_*).
 * Per point it stores the table index
 *     idx = clamp(floor((v - v_min)/dv + 1/2), 0, N_G - 1),
 *     v = c/(f h) on the G axis, v = (f h)/c on the 1/G axis
 * (binary64, no contraction, f h formed first; bit-identical to the same
 * formula on any IEEE machine) and keeps the velocity; the coefficients are
 * rebuilt from them by the recompute kernels.  With HELM27_EXTEND_TABLE and
 * rows outside the table, the operator builds its own wider table on the same
 * axis grid (v_min - k dv .. v_max + k' dv, same lambda, angles, smoother;
 * the first abscissa stays > 0 on the G axis and >= 0 on the 1/G axis) over
 * the model's range, so no row clamps (helm27_op_info reports the axis,
 * helm27_op_table_weights the weights).  Errors: EINVAL (dims < 3, h or
 * freq <= 0, npml too large for the grid, non-positive velocity,
 * HELM27_EXTEND_TABLE with a table not made by helm27_build_table), ERANGE
 * (a widened table would need more than 65535 entries), ENOMEM, EDEVICE. */
int helm27_assemble(helm27_ctx* ctx, const helm27_table* t, const float* vel,
                    int nx, int ny, int nz, double h, double freq,
                    const helm27_pml* pml, int flags, helm27_op** out);
int helm27_op_info(const helm27_op* op, helm27_op_desc* out);
/* Weights of the table the operator uses, host [n_g][7] (as
 * helm27_table_weights).  Errors: EINVAL. */
int helm27_op_table_weights(const helm27_op* op, double* w7);
void helm27_op_destroy(helm27_op* op);

/* Table index of every point with no allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It computes what helm27_assemble stores
 * per point -- idx = clamp(floor((c/(f h) - g_min)/dG + 1/2), 0, N_G - 1),
 * binary64, no contraction, bit-identical to helm27_assemble's index -- for
 * `n` velocities `vel` (device pointer on ctx's device, float32) into `idx`
 * (device pointer on ctx's device, uint16 [n], caller-owned), enqueued on
 * `stream` (NULL = null stream).  Its kernels keep their partial counts in a
 * file-scope device array of the library (131 KB per device, 4096 records of
 * 65536 points), so n is limited to 268,435,456 points (EINVAL beyond).
 * Calls that overlap on one device (any streams, any threads) share that
 * array and race: serialise them.  With `stats` non-NULL the call waits for
 * the stream and fills it (clamped points, invalid velocities -- zero,
 * negative, infinite or NaN -- and the model's G range) and returns EINVAL if
 * any velocity is invalid; with stats NULL it returns right after enqueueing
 * and does not validate.  Errors: EINVAL (null or non-device pointer, n out
 * of range, h or freq not positive, invalid velocities), EDEVICE. */
typedef struct {
    int64_t n_clamped;      /* points whose G fell outside the table (clamped) */
    int64_t n_invalid;      /* velocities that are not finite and positive */
    double  g_min_model;    /* smallest / largest G = c/(f h) of the valid velocities */
    double  g_max_model;
} helm27_index_stats;
int helm27_select_index_noalloc(helm27_ctx* ctx, const helm27_table* t, const float* vel, int64_t n,
                                double h, double freq, uint16_t* idx, helm27_index_stats* stats,
                                void* stream);

/* Test hooks.  helm27_export_index copies the table index of every point to
 * host memory `idx` [N] (uint16).  helm27_export_csr writes the matrix in
 * CSR form to host memory: indptr [N+1], indices [nnz] (ascending columns,
 * nnz = prod(3 n_a - 2)), vals [2 nnz] interleaved complex128; the values
 * are evaluated on the device in FP64.  Pass NULL for indptr to get only
 * the nnz in *nnz_out.  Errors: EINVAL, ENOMEM, EDEVICE. */
int helm27_export_index(const helm27_op* op, uint16_t* idx);
int helm27_export_csr(const helm27_op* op, int64_t* nnz_out, int64_t* indptr,
                      int64_t* indices, double* vals);

/* ---- (b) apply ------------------------------------------------------------
 * y = A u for nrhs right-hand sides (Sec. 2.1, [M + S] p); u and y are device
 * pointers to [nrhs][N] complex values of `dtype` (HELM27_C64: FP32 with FP32
 * accumulation; HELM27_C128: FP64), u and y must not overlap.  `variant`
 * selects HELM27_RECOMPUTE or HELM27_STORED (needs the matching STORE flag at
 * assembly).  Enqueued on `stream` (hipStream_t; NULL = null stream);
 * returns without synchronising.  Errors: EINVAL, EDEVICE. */
int helm27_apply(helm27_op* op, const void* u, void* y, int nrhs, int dtype, int variant,
                 void* stream);

/* Batched apply of several operators (the same product y_i = A_i u_i as
 * helm27_apply with HELM27_RECOMPUTE, Sec. 2.1) in fused launches: the small
 * grids of concurrent requests share one launch of the stencil kernel (up to
 * 8 operators per launch; operators that differ in attenuation, GAm per-row
 * weights or mass form go in separate launches).  ops[n_ops]: operators of
 * one device; u[i], y[i]: device pointers to [nrhs[i]][N_i] complex values
 * of `dtype` (HELM27_C64 or HELM27_C128); nrhs[i] = 0 skips operator i; all
 * arrays are host arrays owned by the caller.  Outputs must not overlap any
 * input or each other.  The tile shape is the small-grid one (per-wavefront
 * tiles, automatic z chunks) whatever helm27_set_tuning chose.  Enqueued on
 * `stream`; returns without synchronising.  Errors: EINVAL (null pointers,
 * n_ops < 0, nrhs[i] < 0, a grid too large for 32-bit vector offsets or
 * whose table slice does not fit in LDS), EDEVICE. */
int helm27_apply_many(helm27_op* const* ops, int n_ops, const void* const* u, void* const* y,
                      const int* nrhs, int dtype, void* stream);

/* Tuning of the recompute kernel's tile shape (output rows per wavefront in
 * the unstretched box, 1..4; more rows reuse more loaded data, fewer rows
 * leave registers for more wavefronts in flight).  helm27_set_tuning sets
 * it for one precision; helm27_tune times every rows choice with each z
 * chunk in {automatic, 8, 16, 32, 64} (helm27_set_zchunk) and kernel
 * variants 0 and 2 (helm27_set_kernel_variant) on the operator with nrhs
 * zero right-hand sides (device scratch allocated and freed inside), keeps
 * the fastest and returns its rows in *best_rows (may be NULL).  Until one
 * of helm27_set_tuning, helm27_tune, helm27_set_kernel_variant or
 * helm27_set_zchunk is called, every launch chooses its own shape from its
 * work size: 2^23 or more point-RHS pairs take variant 2 with 1 row and
 * 32-plane chunks (one RHS) or 2 rows (FP32) and 16-plane chunks (several),
 * smaller launches
 * variant 0 with 2 rows (FP32) / 1 row (FP64) and automatic chunks.  After
 * such a call the operator keeps its explicit settings (operators of 2^23
 * points or more start from variant 2, 1 row, 16-plane chunks; smaller ones
 * from variant 0, 2 / 1 rows, automatic chunks).  Every choice computes the same sums per output; the compiler may
 * fuse multiply-adds differently per choice, so results agree to rounding
 * (not bit for bit) across choices, and bit for bit across runs of one
 * choice.
 * Errors: EINVAL, ENOMEM, EDEVICE. */
int helm27_set_tuning(helm27_op* op, int dtype, int rows_per_wave);
int helm27_tune(helm27_op* op, int nrhs, int dtype, void* stream, int* best_rows);
/* Kernel family of the recompute stencil: 0 = one wavefront per tile, box and
 * PML frame in one launch (default); 1 = LDS-tiled blocks (one block per
 * 64 x 8 or 16 x 16 column tile); 2 = as 0, with the box tiles in groups of
 * 16 (FP32) or 8 (FP64) stacked tiles per block, one per wavefront, that
 * share their plane rows through LDS.
 * All compute the same operator.  Switches off the per-launch choice (see
 * helm27_tune).  Errors: EINVAL. */
int helm27_set_kernel_variant(helm27_op* op, int variant);
/* Constant-Q attenuation of the medium: k^2 = omega^2 / c~^2 with the complex
 * velocity c~ = c (1 - i/(2Q)) (exp(-i omega t): outgoing waves decay), for
 * every later apply, residual and solve of the operator (its stored
 * coefficients are refilled, its multigrid hierarchy rebuilt; the table
 * index and the PML keep the real velocity).  Q = 0 or infinite: none.
 * Errors: EINVAL (Q negative or NaN), EDEVICE. */
int helm27_set_attenuation(helm27_op* op, double Q);
/* Right-hand sides per box wavefront of the FP32 recompute kernels: with
 * nb = 2 or 4 a wavefront computes one output row (62 columns) of nb
 * consecutive right-hand sides at once (block tiles of 16 wavefronts that
 * share plane rows through LDS), so a point's table index, velocity and
 * coefficients are read and formed once per nb right-hand sides; nb = 1 or
 * 0 (default) keep one right-hand side per wavefront.  Used by every mode
 * (apply, residual, Jacobi sweeps) of FP32 launches with several right-hand
 * sides; helm27_tune sweeps it for nrhs >= 2.  Results agree to rounding
 * across choices.  Errors: EINVAL (nb not 0, 1, 2 or 4). */
int helm27_set_rhs_block(helm27_op* op, int nb);
/* Work-item order of launches with several right-hand sides: 2 = right-hand
 * side slowest (each right-hand side's tiles run together, so the rows and
 * planes neighbouring tiles share are re-read from cache), 1 = right-hand
 * side fastest (a tile's right-hand sides run together and share its
 * per-point data), 0 (default) = 2.  helm27_tune sweeps it for nrhs >= 2.
 * Results are bit-identical across orders.  Errors: EINVAL. */
int helm27_set_rhs_order(helm27_op* op, int order);
/* z planes per work item of the wavefront kernel (each item marches its
 * chunk of planes; two extra planes are read per chunk): 0 = automatic
 * (about 4096 work items, 2..16 planes each), else 2..4096.  Results agree
 * to rounding across choices.  Switches off the per-launch choice (see
 * helm27_tune).  Errors: EINVAL. */
int helm27_set_zchunk(helm27_op* op, int zchunk);

/* ---- (c) solve ------------------------------------------------------------ */
typedef struct {
    double tol;          /* relative residual ||b - A u|| / ||b|| per RHS (default 1e-6) */
    int    restart;      /* GMRES(m) restart length, 1..63 (default 28) */
    int    max_inner;    /* Arnoldi steps per refinement step (default 600) */
    int    max_outer;    /* FP64 refinement steps (default 10) */
    double inner_tol;    /* relative reduction asked of each inner solve (default 1e-3) */
    int    precision;    /* HELM27_C64: FP32 inner + FP64 refinement (default);
                            HELM27_C128: everything in FP64 */
    int    mg_levels;    /* multigrid levels, 1..8; -1 (default) = halve while the coarser
                            grid keeps >= 8192 points (4 levels for 400x400x200, 3 for
                            101^3, 2 for 41^3); 0 = no preconditioner */
    double mg_shift;     /* imaginary part b of the preconditioner's mass factor a + i b (default 1.0) */
    int    mg_pre, mg_post;   /* damped-Jacobi sweeps per level before / after the coarse correction (default 2, 1) */
    double mg_omega;     /* Jacobi damping (default 0.6) */
    int    mg_coarse_sweeps;  /* sweeps on the coarsest level (default 3) */
    int    use_graph;    /* replay each multigrid V-cycle from one captured hipGraph
                            (captured on first use, kept with the workspace; the
                            same kernels as the eager launches, so the same
                            results); 0 = eager launches (default 1) */
    int    verbose;
    double mg_shift_re;  /* real part a of the preconditioner's mass factor (default 0) */
    int    reorth_always;/* 1: second classical Gram-Schmidt pass at every Arnoldi step;
                            0 (default): per right-hand side only when the first pass
                            leaves less than 1/sqrt(2) of the vector's norm */
    int    mg_coarse_table; /* weights of the coarse levels, whose rows have G = c/(f 2^l h):
                            0 (default) = the operator's table, clamped at its ends (the
                            clamped rows are counted in the stats); 1 = each level gets a
                            table widened for its own G range (needs a table made by
                            helm27_build_table).  Measured: below about 2.5 points per
                            wavelength the dispersion-fitted weights make the shifted
                            coarse operators a poor correction and GMRES stagnates
                            (201x201x101 at 8 Hz: 811 steps with 0, no convergence in
                            30000 with 1) */
    int    transpose;    /* 1: solve the transposed system A^T u = b (adjoint problems of
                            waveform inversion, Sec. 1) with A^T applied from the stored
                            coefficients (assemble with HELM27_STORE_C128, and also
                            HELM27_STORE_C64 for the mixed precision; else EINVAL); the
                            preconditioner is the multigrid of A, whose rows differ from
                            A^T's only where the weights vary between neighbours */
} helm27_solve_opts;

typedef struct {
    int    outer_iters;
    int    inner_iters;      /* total Arnoldi steps (all refinement steps) */
    int    converged;        /* 1 if every RHS reached tol */
    double max_relres;       /* max over RHS of the FP64 relative residual */
    double seconds;          /* wall time of the call */
    int    mg_levels;        /* multigrid levels of the preconditioner (1: none coarse) */
    int64_t coarse_clamped;  /* coarse-level rows whose G = c/(f 2^l h) fell outside their table */
    int    coarse_tables;    /* coarse levels that use a table widened for their own G range */
    double inner_est;        /* last inner GMRES solve: its Givens (Hessenberg least-squares)
                                estimate of the residual it leaves, relative to its right-hand
                                side, max over RHS (a check of the Arnoldi recurrence: with one
                                FP64 refinement step it equals max_relres to rounding) */
} helm27_solve_stats;

/* Fill `opts` with the defaults above. */
void helm27_solve_opts_default(helm27_solve_opts* opts);

/* Solve A u = b for point sources (Sec. 3.1: s = delta(x - x_s), i.e.
 * amp / h^3 at the source node).  `src` is host memory [nrhs][5] doubles
 * (i, j, k, amp_re, amp_im); every source must lie inside the grid and outside
 * the PML (else ERANGE).  `u` is a device pointer to [nrhs][N] complex128 that
 * receives the solution (its input value is ignored).  On ENOCONV u holds the
 * best iterate and stats says how far it got.  Synchronises `stream` before
 * returning.  Errors: EINVAL, ERANGE, ENOCONV, ENUMERIC, ENOMEM, EDEVICE. */
int helm27_solve(helm27_op* op, const double* src, void* u, int nrhs,
                 const helm27_solve_opts* opts, helm27_solve_stats* stats, void* stream);

/* Several operators solved at once -- typically one model at several
 * frequencies (waveform inversion proceeds frequency by frequency, Sec. 1):
 * ops[k] (distinct operators) with its point sources src[k] (host
 * [nrhs[k]][5], as helm27_solve) into u[k] (device [nrhs[k]][N_k]
 * complex128).  Each solve runs from its own host thread on its own stream,
 * so the frequencies' kernels overlap on the device; each result is
 * bit-identical to the same solve alone.  stats: [nops] or NULL.  Returns
 * OK, ENOCONV if any solve stopped short of the tolerance, or the first
 * other error.  Synchronises before returning.  Errors: EINVAL (null
 * pointers, a repeated operator), ERANGE, ENUMERIC, ENOMEM, EDEVICE. */
int helm27_solve_many(helm27_op* const* ops, int nops, const double* const* src, const int* nrhs,
                      void* const* u, const helm27_solve_opts* opts, helm27_solve_stats* stats);

/* Same with a general right-hand side: `b` device pointer [nrhs][N]
 * complex128 (the Xi-scaled system's right-hand side). */
int helm27_solve_rhs(helm27_op* op, const void* b, void* u, int nrhs,
                     const helm27_solve_opts* opts, helm27_solve_stats* stats, void* stream);

/* ---- serving ----------------------------------------------------------------
 * A request loop on the context: requests (a velocity model, a frequency, point
 * sources) arrive at any time; each is admitted when a slot is free and its
 * estimated device footprint (operator + multigrid hierarchy + Krylov
 * workspace) fits in the context's HBM budget next to the requests already
 * running.  Admitted requests run concurrently, each on its own HIP stream, so
 * their kernels overlap on the device; all right-hand sides of a request are
 * solved together by the multi-RHS kernels, unless together they would need
 * more than half the budget: then the request is solved in chunks of the
 * largest right-hand-side count that fits in half the budget, one after
 * another on one operator (its stats: the chunks' total steps and seconds,
 * the worst residual, converged only if every chunk did).  Operators and their multigrid
 * hierarchies stay resident in a cache keyed by (model_key, grid, h, f, PML)
 * for later requests on the same model.  Timestamps are seconds on the host's
 * steady clock. */
typedef struct {
    int    max_slots;            /* requests running at once (default 4) */
    helm27_solve_opts solve;     /* solver options of every request */
    double table_gmin, table_gmax, table_dg, table_lambda;   /* table built at start (2.5, 60, 0.05, 1e-3) */
    int    max_cached_ops;       /* resident operators kept for reuse (default 8) */
    int    max_chunk_rhs;        /* cap on right-hand sides per solve (0: by footprint only) */
} helm27_serve_opts;

typedef struct {
    const float*  vel;           /* [nz][ny][nx] float32, host or device; copied at submit */
    int           nx, ny, nz;
    double        h, freq;
    helm27_pml    pml;
    const double* src;           /* host [nrhs][5] (i, j, k, amp_re, amp_im); copied at submit */
    int           nrhs;
    uint64_t      model_key;     /* same key = same velocity model (0: never reuse) */
    void*         out;           /* device [nrhs][N] complex128, caller-owned, written at completion */
} helm27_request;

typedef struct {
    int    status;               /* HELM27_OK / ENOCONV / ... of the solve */
    helm27_solve_stats stats;
    double t_submit, t_start, t_done;
} helm27_result;

void helm27_serve_opts_default(helm27_serve_opts* opts);
/* Start the loop (builds the weight table once).  Errors: EINVAL (already
 * started, bad options), ENOMEM. */
int helm27_serve_start(helm27_ctx* ctx, const helm27_serve_opts* opts);
/* Queue a request; returns a ticket.  Errors: EINVAL (bad request or not
 * started), EADMIT (even one right-hand side exceeds the HBM budget), ERANGE
 * (a source outside the grid or in the PML). */
int helm27_serve_submit(helm27_ctx* ctx, const helm27_request* req, uint64_t* ticket);
/* Result of a ticket: HELM27_OK with *res filled when done, HELM27_EAGAIN while
 * queued or running, HELM27_ENOTFOUND for an unknown ticket. */
int helm27_serve_poll(helm27_ctx* ctx, uint64_t ticket, helm27_result* res);
/* Block until the ticket is done or timeout_s elapses (EAGAIN). */
int helm27_serve_wait(helm27_ctx* ctx, uint64_t ticket, helm27_result* res, double timeout_s);
/* Finish every submitted request, then stop the workers and free the cache. */
int helm27_serve_stop(helm27_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* HELM27_H */
