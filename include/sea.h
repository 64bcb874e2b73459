/*
 * sea.h - C ABI of the MI355X (gfx950) library for the exact-exchange action
 * on localized orbitals and the ACE low-rank build (the "exx" and "decomp"
 * steps of the SeA approach, arXiv 2208.06097).
 *
 * Conventions used by every call
 *   - Grid: periodic orthorhombic cell of n[0] x n[1] x n[2] points, spacing
 *     h[a] = L[a]/n[a], point (ix,iy,iz) at (ix*h0, iy*h1, iz*h2), x fastest.
 *   - Orbital arrays (phi, W, xi, psi) are orbital-major device arrays:
 *     element (k, iz, iy, ix) at k*Ng + (iz*n1 + iy)*n0 + ix, Ng = n0*n1*n2.
 *   - Inner product <f,g> = dV * sum f g, dV = h0*h1*h2 (grid quadrature).
 *   - Atomic units (hartree, bohr); Poisson equation Lap v = -4 pi rho.
 *   - Device pointers are plain HIP device addresses owned by the caller; the
 *     library never frees them and allocates no device memory on the exx or
 *     ACE paths: scratch space is the caller's workspace, sized by the
 *     *_workspace_bytes calls.
 *   - All device work is enqueued on opts.hip_stream (NULL = default stream).
 *     A call blocks the host only when it returns host results (exx_host,
 *     stats_host, loss_host, failed_pivot).
 *   - Every call returns sea_status: 0 = OK, > 0 = warning (outputs written),
 *     < 0 = error (nothing reliable written).  sea_last_error() gives the
 *     context's last message.  Arguments are validated before any launch.
 */
#ifndef SEA_H
#define SEA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SEA_OK = 0,
    SEA_W_NOT_CONVERGED = 1, /* some pair hit max_iter; outputs still written */
    SEA_W_EIGEN_FALLBACK = 2,/* Mbar not positive definite: the eigen scheme of
                              * App. A was used instead of Cholesky             */
    SEA_E_ARG = -1,          /* invalid argument (message says which)          */
    SEA_E_HIP = -2,          /* HIP runtime error                               */
    SEA_E_NOMEM = -3,        /* workspace smaller than *_workspace_bytes        */
    SEA_E_NOT_PD = -4,       /* symmetrized M not positive definite (ACE)       */
    SEA_E_NONFINITE = -5,    /* NaN/Inf in an input or a reduction              */
    SEA_E_RANK = -6          /* Phi^T has rank < n_occ (SCDM pivoted QR)        */
} sea_status;

typedef enum { SEA_F64 = 0, SEA_F32 = 1, SEA_BF16 = 2 } sea_dtype;

/* Initial guess of each pair's CG solve.  The stopping rule (relative true
 * residual) does not depend on the start. */
typedef enum {
    SEA_START_ZERO = 0,      /* x0 = 0                                          */
    SEA_START_MULTIPOLE = 1, /* x0 = regularized multipole potential (Eq. 10)   */
    SEA_START_LEARNED = 2,   /* x0 from the 3-D convolutional network (attached) */
    SEA_START_SPECTRAL = 3   /* multipole start plus the correction from a fast */
                             /* sine-transform solve of b - A x0 with the same  */
                             /* stencil continued oddly past the faces (domains */
                             /* with every axis <= 64; others keep the          */
                             /* multipole start)                                */
} sea_start;

typedef struct {
    int32_t n[3];
    double L[3];
} sea_grid;

/* Low-rank decomposition of Mbar in the ACE build (Eq. 18, App. A). */
typedef enum {
    SEA_DECOMP_CHOLESKY = 0, /* Mbar = L L^T; a non-positive pivot is an error   */
    SEA_DECOMP_EIGEN = 1,    /* Mbar = Q Lambda Q^T, zeta = W Q |Lambda|^{-1/2}  */
    SEA_DECOMP_AUTO = 2      /* Cholesky, the eigen scheme if Mbar is not PD     */
} sea_decomp;

/* One kept orbital pair <ij> (Sec. II.B): i <= j, and its truncated domain,
 * the box of n[0] x n[1] x n[2] interior points starting at grid index lo[]
 * (lo may be negative or beyond the cell: indices wrap periodically), plus
 * the multipole origin (bohr, unwrapped coordinates). */
typedef struct {
    int32_t i, j;
    int32_t lo[3];
    int32_t n[3];
    double origin[3];
} sea_pair;

typedef struct {
    int32_t fd_half_order;  /* 6: O(h^12) Laplacian (App. C); only 6 accepted  */
    int32_t lmax;           /* 6: multipole order (App. C); 0..6 accepted      */
    double rel_tol;         /* CG stop: |b - A x|_2 <= rel_tol |b|_2           */
    int32_t max_iter;       /* CG iteration cap per pair                       */
    sea_dtype stencil_dtype;/* CG state precision: SEA_F64 or SEA_F32          */
    sea_dtype ace_dtype;    /* xi / K psi GEMM inputs: F64, F32 or BF16        */
    sea_start start;        /* CG initial guess                                */
    int32_t cg_variant;     /* F32 state: z-march kernel variant; -1 = the     */
                            /* context's autotuned choice, else the default;  */
                            /* 0..sea_cg_variant_count()-1 = that variant     */
    int32_t profile;        /* non-zero: time each stage with HIP events       */
    sea_dtype nn_weight_dtype; /* learned start: network weights F32 or BF16   */
    void *hip_stream;       /* hipStream_t; NULL = default stream              */
    sea_decomp ace_decomp;  /* ACE decomposition (default Cholesky)            */
    double cg_xc_beta_min;  /* paired-update CG variants (-xc): smallest      */
                            /* beta_{k-1} for which a pending step is         */
                            /* recovered from p_k and r_k, else it is written */
                            /* by a separate pass; 0 selects 0.25; >= 0       */
} sea_opts;

/* Stages timed when opts.profile is set (indices into sea_stage_times). */
typedef enum {
    SEA_STAGE_GATHER = 0,   /* pair density, b = 4 pi rho, multipole moments   */
    SEA_STAGE_BOUNDARY = 1, /* multipole boundary values folded into b         */
    SEA_STAGE_GUESS = 2,    /* initial guess (multipole or learned start)      */
    SEA_STAGE_CG = 3,       /* CG solves (the hot loop; one kernel launch)     */
    SEA_STAGE_SCATTER = 4,  /* W accumulation                                  */
    SEA_STAGE_ENERGY = 5,   /* E_xx reduction                                  */
    SEA_STAGE_ACE_M = 6,    /* M = dV Phi^T W and symmetrization               */
    SEA_STAGE_ACE_CHOL = 7, /* Cholesky and L^{-1}                             */
    SEA_STAGE_ACE_XI = 8,   /* xi = W L^{-T}                                   */
    SEA_STAGE_ACE_APPLY = 9,/* K psi                                           */
    SEA_STAGE_FINISH = 10,  /* FP32 state: e_ij (from the scatter's partials   */
                            /* when W is formed) and the flags per pair        */
    SEA_STAGE_SCDM = 11,    /* SCDM pivoted QR, P_CC^{-1/2} and U              */
    SEA_STAGE_ROTATE = 12,  /* orbital rotation by U or U^{-1}                 */
    SEA_STAGE_DST = 13,     /* spectral start: the three sine-transform passes */
                            /* (inside the GUESS stage)                        */
    /* single kernels of the spectral start (inside the stages above)          */
    SEA_STAGE_DST_PLANE_FWD = 14, /* k_dst_plane, forward 2-D transforms       */
    SEA_STAGE_DST_ZLINE = 15,     /* k_dst_zline, z transforms and division    */
    SEA_STAGE_DST_PLANE_INV = 16, /* k_dst_plane, inverse 2-D transforms       */
    SEA_STAGE_RESIDUAL = 17,      /* k_residual_zm: FP64 b - A x of the start  */
    SEA_STAGE_FACE = 18,          /* x0 and -D x0 on the face points           */
    SEA_STAGE_FOLD = 19,          /* multipole ghost values folded into b      */
    SEA_STAGE_COUNT = 20
} sea_stage;

/* Per-pair diagnostics (Eq. 8 and Eq. 17 quantities on the pair domain). */
typedef struct {
    int32_t iters;          /* CG iterations                                   */
    int32_t converged;      /* 1 if the true residual met rel_tol              */
    double rel_res;         /* final true relative residual                    */
    double e_ij;            /* dV sum rho_ij v_ij                              */
    double s_abs;           /* dV sum |rho_ij|  (Eq. 17)                       */
    double q;               /* dV sum rho_ij (pair charge)                     */
} sea_pair_stat;

typedef struct sea_ctx sea_ctx;

/* Library version string (static storage). */
const char *sea_version(void);

/* Fill *o with the defaults: half order 6, lmax 6, rel_tol 1e-8,
 * max_iter 10000, F64 stencil and ACE, zero start, cg_variant -1,
 * BF16 network weights, profiling off. */
void sea_opts_default(sea_opts *o);

/* Create a context on the current HIP device.  The context owns only host
 * state (options, error text, tuning cache, network weights).  Errors:
 * SEA_E_ARG for a NULL out pointer or unsupported options, SEA_E_HIP when no
 * gfx950 device is current. */
sea_status sea_create(const sea_opts *opts, sea_ctx **out);
sea_status sea_destroy(sea_ctx *ctx);
const char *sea_last_error(const sea_ctx *ctx);
/* Replace the options of an existing context (validated as in sea_create). */
sea_status sea_set_opts(sea_ctx *ctx, const sea_opts *opts);

/* Pair selection and pair domains (Sec. II.B), host only.  Keeps (i <= j)
 * when the minimum-image distance |c_j - c_i| < r_pair (self pairs always);
 * the domain is the cube of w = ceil(half_width/h) points on each side of the
 * grid point nearest to the minimum-image midpoint c_i + (c_j - c_i)/2
 * (floor(m/h + 0.5) per axis, not wrapped), and the multipole origin is that
 * grid point.  Pairs are written in (i, j) lexicographic order.
 * centers_host: n_occ x 3 doubles.  Returns SEA_E_NOMEM (with *n_out set to
 * the full count) when cap is too small. */
sea_status sea_build_pairs(const sea_grid *grid, int n_occ, const double *centers_host,
                           double r_pair, double half_width, sea_pair *out, int cap,
                           int *n_out);

/* The paper's own truncation (Sec. II.B, Eq. 16-17), device part.  Each
 * orbital's box Omega_ii holds >= 1 - eps of |phi_i|^2: per axis, the
 * shortest cyclic run of grid indices whose marginal mass is >= (1 - eps/3)
 * of the total (ties: largest mass, then smallest start), so the mass
 * outside the product box is <= eps.  Pair boxes are Omega_ii intersect
 * Omega_jj per axis (the longer piece if the runs overlap twice); a pair
 * (i <= j) is kept when its box is non-empty and
 * S_ij = dV sum_box |phi_i phi_j| >= delta (Eq. 17; the paper derives delta
 * from eps elsewhere, the caller chooses it here).  The box written out, on
 * which rho_ij is taken and the Poisson equation solved, is Omega_ij grown
 * by `pad` >= 0 points on each side (at most the cell per axis), which moves
 * the multipole boundary away from the pair density.  Output in (i, j)
 * order: lo = box start (boxes may run past the cell edge and wrap), n = box
 * extents, origin = box centre (lo + (n - 1)/2) h.  s_out (nullable)
 * receives S_ij (over the unpadded Omega_ij).  dbox_out (nullable, 12 int32
 * per pair) receives the paper's Omega^D boxes for sea_cell.dbox_host: for
 * W_i the box of phi_j (i != j) or Omega_ii doubled about its centre
 * (i == j, at most the cell), for W_j the box of phi_i, each shifted by a
 * multiple of the cell to lie nearest the pair's domain and grown to cover
 * that domain (so W takes the pair wherever e_ij does; at most the cell).  phi_dev:
 * n_occ x Ng, F64 or F32.  Synchronizes.  SEA_E_NOMEM with *n_out = full
 * count when cap is too small. */
sea_status sea_eps_workspace_bytes(sea_ctx *ctx, const sea_grid *grid, int n_occ, size_t *bytes);
sea_status sea_build_pairs_eps(sea_ctx *ctx, const sea_grid *grid, int n_occ, const void *phi_dev,
                               sea_dtype phi_dtype, double eps, double delta, int pad, void *ws_dev,
                               size_t ws_bytes, sea_pair *out, double *s_out, int32_t *dbox_out, int cap,
                               int *n_out);

/* Device workspace needed by sea_exx_action / sea_exx_pair_solve for this
 * pair list (bytes, 256-byte aligned). */
sea_status sea_exx_workspace_bytes(sea_ctx *ctx, const sea_grid *grid, int n_occ, int n_pairs,
                                   const sea_pair *pairs_host, size_t *bytes);

/* The V_xx action on localized orbitals (Eq. 8-14): for every pair, the pair
 * density rho_ij = phi_i phi_j on its domain (wrapped indices), its multipole
 * moments (Eq. 11, l <= lmax), boundary values on the ghost layers the
 * stencil reaches (Eq. 10), the CG solve of -Lap_h v = 4 pi rho (Eq. 9) to
 * the relative true residual rel_tol, then
 *     W_i = sum_{j in <ij>} v_ij phi_j  on the pair domains (Eq. 14),
 *     E_xx = -sum_i e_ii - 2 sum_{i<j} e_ij  (Eq. 8 over ordered pairs).
 * phi_dev: n_occ x Ng of phi_dtype (SEA_F64 or SEA_F32).  W_dev: n_occ x Ng
 * FP64, overwritten.  exx_dev: device FP64 scalar (nullable).  exx_host and
 * stats_host (n_pairs entries) are nullable; when given the call syncs the
 * stream.  The scatter is owner-computes in pair order: W is bit-identical
 * run to run.  Returns SEA_W_NOT_CONVERGED if any pair hit max_iter. */
sea_status sea_exx_action(sea_ctx *ctx, const sea_grid *grid, int n_occ, const void *phi_dev,
                          sea_dtype phi_dtype, int n_pairs, const sea_pair *pairs_host,
                          void *ws_dev, size_t ws_bytes, double *W_dev, double *exx_dev,
                          double *exx_host, sea_pair_stat *stats_host);

/* One cell of a batched call (pairs of every cell are solved together in
 * one persistent launch; cells may differ in grid, orbitals and pairs).
 * phi_dev, W_dev and exx_dev are caller-owned device buffers as in
 * sea_exx_action; exx_dev is nullable. */
typedef struct {
    sea_grid grid;
    int32_t n_occ;
    sea_dtype phi_dtype;
    const void *phi_dev;
    int32_t n_pairs;
    const sea_pair *pairs_host;
    double *W_dev;
    double *exx_dev;
    /* Nullable: n_pairs x 12 int32, for pair k the box where W_i takes v_ij
     * phi_j (lo[3], n[3]) and then the box where W_j takes v_ij phi_i, both in
     * the unwrapped frame of the pair's domain; v_ij outside the domain is the
     * multipole potential (Eq. 10).  This is the paper's Omega^D (end of
     * Sec. II.B); sea_build_pairs_eps writes it.  NULL: both boxes are the
     * pair's domain (Eq. 13-14 on the domain). */
    const int32_t *dbox_host;
} sea_cell;

/* Workspace for sea_exx_action_batched / a plan over these cells. */
sea_status sea_exx_batched_workspace_bytes(sea_ctx *ctx, int n_cells, const sea_cell *cells, size_t *bytes);

/* The V_xx action of every cell (same definition as sea_exx_action), all
 * pairs of all cells in one queue: one persistent CG launch for the whole
 * batch.  Per cell W_dev and exx_dev are written; exx_host (n_cells,
 * nullable) and stats_host (sum of n_pairs, in cell order, nullable) make
 * the call synchronize.  Results are bit-identical to per-cell calls. */
sea_status sea_exx_action_batched(sea_ctx *ctx, int n_cells, const sea_cell *cells, void *ws_dev,
                                  size_t ws_bytes, double *exx_host, sea_pair_stat *stats_host);

/* Kernel variants of the FP32-state CG solve (workgroup size, prefetch of
 * the output plane, planes in flight).  Names are static strings; NULL for an
 * index out of range. */
int sea_cg_variant_count(void);
const char *sea_cg_variant_name(int variant);

/* Autotuner for the FP32-state CG solve (the batching workload's tile and
 * schedule choice): runs the CG of a strided sample of `sample_pairs` pairs
 * of these cells (zero start, exactly `iters` iterations each, so every
 * variant does the same work) once per variant, times each launch with HIP
 * events, and keeps the fastest as the context's choice (used while
 * opts.cg_variant is -1).  ms_host (sea_cg_variant_count() floats, nullable)
 * receives the times and *best the chosen index.  The workspace must hold
 * sea_exx_batched_workspace_bytes of the same cells; W_dev may be NULL.
 * Synchronizes.  SEA_E_ARG for cells that the FP32 state cannot run (grids
 * not cubic, domains wider than 64 points in x or y). */
sea_status sea_exx_autotune(sea_ctx *ctx, int n_cells, const sea_cell *cells, void *ws_dev, size_t ws_bytes,
                            int sample_pairs, int iters, float *ms_host, int *best);

/* Kernel variants of the spectral start's sine-transform passes (one plane
 * kernel and one z-line kernel per call): workgroups per pair and how a
 * tile is staged; every variant computes the same sums in the same order,
 * so results do not depend on the choice.  Indices 0 .. count-1: the plane
 * variants first, then the z-line ones (a name starting "plane-" or
 * "zline-"); NULL out of range. */
int sea_spectral_variant_count(void);
const char *sea_spectral_variant_name(int variant);
/* Fixes the variants a context uses (plane: index among the plane
 * variants, zline: index among the z-line variants; -1: the autotuner's
 * choice, else the first).  SEA_E_ARG out of range. */
sea_status sea_set_spectral_variants(sea_ctx *ctx, int plane, int zline);
/* Schedules of the owner-computes scatter of W (Eq. 13-14): the order in
 * which its (orbital, tile) workgroups run, which sets what the GPU's L2
 * caches share; every variant computes the same sums in the same order, so
 * results do not depend on the choice.  Names for 0 .. count-1, NULL out of
 * range. */
int sea_scatter_variant_count(void);
const char *sea_scatter_variant_name(int variant);
/* Fixes the scatter schedule of a context (-1: the autotuner's choice,
 * else the first).  SEA_E_ARG out of range. */
sea_status sea_set_scatter_variant(sea_ctx *ctx, int variant);
/* Autotuner of the scatter schedule: for these cells (every pair; pair
 * potentials set to zero in the workspace, which must hold
 * sea_exx_batched_workspace_bytes of the same cells), times one scatter of
 * every variant with HIP events (the second of two launches) and keeps the
 * fastest as the context's choice.  The cells' W_dev (required) are
 * overwritten.  ms_host (sea_scatter_variant_count() floats, nullable)
 * receives the times, *best (nullable) the chosen index.  Synchronizes. */
sea_status sea_scatter_autotune(sea_ctx *ctx, int n_cells, const sea_cell *cells, void *ws_dev, size_t ws_bytes,
                                float *ms_host, int *best);
/* Per-pair residual histories (diagnostics of the Eq. 9 solves).  With
 * hist_dev set, every later exx call of this context writes, for pair k of
 * the call and iteration t = 0 .. len, the relative residual
 * |r_t| / |b| at hist_dev[k * (len + 1) + t] (FP64, device memory owned by
 * the caller, n_pairs * (len + 1) doubles, n_pairs of the call): t = 0 is
 * the start's true FP64 residual, t >= 1 the CG's recursive residual after
 * t iterations (FP32 z-march, FP64 row tiles and their preconditioned form;
 * the generic FP64 kernel records its exit only).  Entries after
 * a pair's last iteration are NaN.  hist_dev NULL or len < 0 turns the
 * recording off.  The buffer must hold the next calls' pairs; it is not
 * checked.  SEA_E_ARG for a negative len with a non-NULL buffer. */
sea_status sea_set_residual_history(sea_ctx *ctx, double *hist_dev, int len);
/* Autotuner of the transform passes (the timed form's schedule choice):
 * on a strided sample of `sample_pairs` pairs of these cells, times the
 * forward plane pass of every plane variant and the z-line pass of every
 * z-line variant with HIP events (the second of two launches), and keeps
 * the fastest of each as the context's choice.  ms_host
 * (sea_spectral_variant_count() floats, nullable) receives the times;
 * *best_plane, *best_zline (nullable) the chosen indices.  The workspace
 * must hold sea_exx_batched_workspace_bytes of the same cells for a context
 * with the spectral start.  Synchronizes. */
sea_status sea_spectral_autotune(sea_ctx *ctx, int n_cells, const sea_cell *cells, void *ws_dev, size_t ws_bytes,
                                 int sample_pairs, float *ms_host, int *best_plane, int *best_zline);

/* A plan fixes the cells, pair tables and workspace once (tables are
 * uploaded at creation) and records the whole kernel sequence of the batched
 * action into a HIP graph; sea_exx_plan_launch replays it on `hip_stream`
 * with no host work and no allocation.  The cells' device buffers and the
 * workspace must stay valid while the plan is used.  sea_exx_plan_results
 * waits for the last launch and copies E_xx per cell and the per-pair stats
 * (both nullable).  Stage profiling is not recorded in a plan. */
typedef struct sea_plan sea_plan;
/* Workspace bytes of a plan of these cells: a plan always runs the kernel
 * sequence a graph can hold, so it needs no arrays of the FP64 row-tile CG
 * (at most sea_exx_batched_workspace_bytes of the same cells). */
sea_status sea_exx_plan_workspace_bytes(sea_ctx *ctx, int n_cells, const sea_cell *cells, size_t *bytes);
sea_status sea_exx_plan_create(sea_ctx *ctx, int n_cells, const sea_cell *cells, void *ws_dev,
                               size_t ws_bytes, sea_plan **out);
sea_status sea_exx_plan_launch(sea_plan *plan, void *hip_stream);
sea_status sea_exx_plan_results(sea_plan *plan, double *exx_host, sea_pair_stat *stats_host);
sea_status sea_exx_plan_destroy(sea_plan *plan);

/* Per-pair potentials without the scatter (same solve as sea_exx_action):
 * v_dev receives, for pair k, its interior potential at offset k*stride
 * doubles (stride = max over pairs of n0*n1*n2 rounded up to a multiple of
 * 32, layout [z][y][x]); Q_dev
 * (nullable) receives 49 real orthonormal multipole moments per pair
 * (index l*l + l + m, Eq. 11 with real Y_lm); e_dev (nullable) e_ij. */
sea_status sea_exx_pair_solve(sea_ctx *ctx, const sea_grid *grid, int n_occ, const void *phi_dev,
                              sea_dtype phi_dtype, int n_pairs, const sea_pair *pairs_host,
                              void *ws_dev, size_t ws_bytes, double *v_dev, double *Q_dev,
                              double *e_dev, sea_pair_stat *stats_host);

/* ACE build (Eq. 18, App. A): M = dV Phi^T W (FP64 matrix cores, FP64
 * accumulation), Mbar = (M + M^T)/2, Mbar = L L^T (FP64 Cholesky, no
 * pivoting), xi = W L^{-T} on the matrix cores with operands in ace_dtype
 * (FP32 accumulation for F32/BF16), stored orbital-major in ace_dtype.
 * With opts.ace_decomp = SEA_DECOMP_EIGEN (or AUTO after a failed pivot):
 * Mbar = Q Lambda Q^T (FP64 Jacobi) and xi = zeta = W Q |Lambda|^{-1/2}
 * (App. A: the imaginary factor of a negative eigenvalue cancels against
 * its conjugate, so K = -W Q |Lambda|^{-1} Q^T W^T), null eigenvalues
 * dropped; L_dev then receives Q |Lambda|^{-1/2} and AUTO returns
 * SEA_W_EIGEN_FALLBACK.  M_dev, L_dev: n_occ x n_occ row-major FP64
 * (L lower, upper triangle zero).  On a non-positive pivot returns
 * SEA_E_NOT_PD and *failed_pivot = 1-based pivot index (0 on success).
 * ws_dev: sea_ace_workspace_bytes bytes. */
sea_status sea_ace_workspace_bytes(sea_ctx *ctx, int64_t n_grid, int n_occ, int n_vec,
                                   size_t *bytes);
sea_status sea_ace_build(sea_ctx *ctx, int64_t n_grid, int n_occ, double dV, const double *phi_dev,
                         const double *W_dev, void *ws_dev, size_t ws_bytes, double *M_dev,
                         double *L_dev, void *xi_dev, int *failed_pivot);

/* K psi = -xi (dV xi^T psi)  (Eq. 18): psi_dev n_vec x n_grid in ace_dtype,
 * out_dev n_vec x n_grid in ace_dtype (FP32 for BF16), xi_dev from
 * sea_ace_build.  Both products run on the matrix cores with operands in
 * ace_dtype: FP64 accumulation for F64, FP32 for F32/BF16 (the K-slice
 * partials of dV xi^T psi are summed in FP64). */
sea_status sea_ace_apply(sea_ctx *ctx, int64_t n_grid, int n_occ, double dV, const void *xi_dev,
                         int n_vec, const void *psi_dev, void *ws_dev, size_t ws_bytes,
                         void *out_dev);

/* Allocation-free K psi, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same product and arguments as sea_ace_apply without the
 * workspace: the library works in a static device array of
 * SEA_NOALLOC_SCRATCH_BYTES that each GPU it runs on holds from module load
 * until the process ends (its address is looked up once per device in
 * sea_create).  It holds C = dV xi^T psi (n_occ x n_vec FP64) and the K-slice
 * partials of that product (at least one slice of n_occ x n_vec FP64, more
 * slices when there is room; the result matches sea_ace_apply to the
 * rounding of a different slicing).  Returns SEA_E_NOMEM when
 * 16 n_occ n_vec bytes exceed the array (n_occ = n_vec = 1448 at most).
 * Enqueued on opts.hip_stream, no host synchronization, no allocation.
 * Every call on one GPU shares the array and it keeps the last call's
 * contents: calls that overlap on one GPU (another stream, another thread,
 * another context) race.  The current device must be the context's. */
#define SEA_NOALLOC_SCRATCH_BYTES (32u << 20)
sea_status sea_ace_apply_noalloc(sea_ctx *ctx, int64_t n_grid, int n_occ, double dV, const void *xi_dev,
                                 int n_vec, const void *psi_dev, void *out_dev);

/* E_xx = -sum_ik <phi_i, xi_k>^2 (Eq. 19): FP64 products (xi of any
 * ace_dtype converts exactly), FP64 result on the host. */
sea_status sea_ace_energy(sea_ctx *ctx, int64_t n_grid, int n_occ, double dV, const double *phi_dev,
                          const void *xi_dev, void *ws_dev, size_t ws_bytes, double *exx_host);

/* Outer-loop convergence by successive idempotency (App. B):
 * dI = 1 - sum_ij <phi_new_i, phi_old_j>^2 / n_occ, the inner products in FP64
 * on the matrix cores.  phi_new_dev, phi_old_dev: n_occ x n_grid FP64.
 * Workspace: sea_ace_workspace_bytes(n_grid, n_occ, 0).  Synchronizes. */
sea_status sea_successive_idempotency(sea_ctx *ctx, int64_t n_grid, int n_occ, double dV,
                                      const double *phi_new_dev, const double *phi_old_dev, void *ws_dev,
                                      size_t ws_bytes, double *dI_host);

/* ---------------------------------------------------------------------
 * SCDM localization (Sec. II.A) and the rotations between orbital sets.
 * --------------------------------------------------------------------- */

/* Workspace of sea_scdm for n_occ orbitals on n_grid points. */
sea_status sea_scdm_workspace_bytes(sea_ctx *ctx, int64_t n_grid, int n_occ, size_t *bytes);

/* Selected columns of the density matrix (Eq. 1-6).  phi_dev: n_occ x
 * n_grid orbital-major (row i = orbital i), phi_dtype F64 or F32, read as
 * the rows of Phi^T.  Eq. 1: column-pivoted QR of Phi^T, pivots only, in
 * FP64 (each pivot is the column whose part orthogonal to the columns
 * already chosen is longest, first grid index on ties); Eq. 3-5 with
 * B = (Phi^T)_{:,C} and P_CC = B^T B (the density matrix at the selected
 * points; X^T X for orbitals orthonormal as grid vectors), so that
 * U = B P_CC^{-1/2} is orthogonal: U is the polar factor of B, computed by
 * the FP64 Newton-Schulz iteration on the matrix cores.
 * Outputs:
 *   U_dev       n_occ x n_occ FP64 row-major, U[j*n_occ + k] = U_jk;
 *   phi_loc_dev (nullable) n_occ x n_grid in phi_dtype, Eq. 6:
 *               phi_loc_k = sum_j phi_j U_jk (FP64 matrix cores for F64,
 *               FP32 for F32); must not overlap phi_dev;
 *   piv_host    (nullable) n_occ int32 grid indices C in pivot order;
 *   rdiag_host  (nullable) n_occ doubles |R_kk|;
 *   rounds_host (nullable) number of passes over Phi^T (pivots are chosen
 *               in rounds: each round ends when the best candidate no
 *               longer provably beats every column outside the candidate
 *               set, then all column norms are brought up to date).
 * n_occ <= 2048, n_grid >= n_occ.  SEA_E_RANK when a residual column
 * norm^2 drops below 1e-26 of the largest initial one, or when the polar
 * iteration has not converged in 120 steps.  ws_dev:
 * sea_scdm_workspace_bytes bytes.  Synchronizes once per round. */
sea_status sea_scdm(sea_ctx *ctx, int64_t n_grid, int n_occ, const void *phi_dev, sea_dtype phi_dtype,
                    void *ws_dev, size_t ws_bytes, double *U_dev, void *phi_loc_dev, int32_t *piv_host,
                    double *rdiag_host, int *rounds_host);

/* Orbital rotation, orbital-major X and Y (n_occ x n_grid, dtype F64 or
 * F32, not overlapping), U from sea_scdm (orthogonal):
 *   inverse = 0:  Y_k = sum_j X_j U_jk             (Eq. 6, into the SCDM set)
 *   inverse = 1:  Y_i = sum_j X_j (U^{-1})_ji      (Eq. 15, back-rotation
 *                 of W or D_xx to the input set; U^{-1} = U^T).
 * Matrix cores, FP64 for F64 and FP32 for F32.  Asynchronous. */
sea_status sea_rotate(sea_ctx *ctx, int64_t n_grid, int n_occ, sea_dtype dtype, const double *U_dev,
                      int inverse, const void *X_dev, void *Y_dev);

/* ---------------------------------------------------------------------
 * Learned CG warm start (an extension of the CG initial guess of Eq. 9; the
 * solve still runs to the same true residual).  A 3-D U-Net (16 channels,
 * levels D, D/2, D/4, D/8, 3x3x3 convolutions with ReLU, average-pool down,
 * nearest up, skip concatenation, 15 convolutions: e0a e0b e1a e1b e2a e2b
 * e3a e3b d2a d2b d1a d1b d0a d0b head) maps x = rho/s resampled to D^3
 * (corner-aligned trilinear, s = dV sum |rho|) to the correction
 * (v - v_ME)/s of the multipole start; the start is v_ME + s up(net(x)).
 * Parameters are one flat FP32 array, per layer weights [O][C][3][3][3] then
 * bias [O].  Activations FP32; weights FP32 or BF16 (opts.nn_weight_dtype),
 * FP32 accumulation.
 * --------------------------------------------------------------------- */

/* Number of FP32 parameters of the network. */
size_t sea_nn_param_count(void);
/* Bytes of the device state: FP32 parameters, their BF16 copy, Adam m, v. */
sea_status sea_nn_state_bytes(sea_ctx *ctx, size_t *bytes);
/* Upload parameters (host FP32, sea_nn_param_count floats), zero the Adam
 * moments and refresh the BF16 copy. */
sea_status sea_nn_set_params(sea_ctx *ctx, void *state_dev, const float *params_host);
/* Download the FP32 parameters (synchronizes). */
sea_status sea_nn_get_params(sea_ctx *ctx, const void *state_dev, float *params_host);
/* Workspace for a batch of `batch` inputs of D^3 (D a multiple of 8, <= 64). */
sea_status sea_nn_workspace_bytes(sea_ctx *ctx, int batch, int D, size_t *bytes);
/* y = net(x); x, y: batch x D^3 FP32 device arrays. */
sea_status sea_nn_forward(sea_ctx *ctx, const void *state_dev, int batch, int D, const float *x_dev,
                          float *y_dev, void *ws_dev, size_t ws_bytes);
/* Inference of the same network on the matrix cores: BF16 weights (the
 * state's BF16 copy) and BF16 activations with FP32 accumulation
 * (v_mfma_f32_16x16x32_bf16), network grid 32^3 only.  x_dev, y_dev:
 * batch x 32^3 floats.  This is what the learned start uses when
 * opts.nn_weight_dtype is SEA_BF16; sea_nn_forward keeps FP32 activations. */
sea_status sea_nn_infer_workspace_bytes(sea_ctx *ctx, int batch, size_t *bytes);
sea_status sea_nn_infer(sea_ctx *ctx, const void *state_dev, int batch, const float *x_dev, float *y_dev,
                        void *ws_dev, size_t ws_bytes);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, `step`
 * 1-based) on the mean squared error between net(x) and t.  loss_host
 * (nullable) receives the loss before the step (synchronizes); grad_dev
 * (nullable, sea_nn_param_count floats) receives the gradient. */
sea_status sea_nn_train_step(sea_ctx *ctx, void *state_dev, int batch, int D, const float *x_dev,
                             const float *t_dev, float lr, int step, void *ws_dev, size_t ws_bytes,
                             double *loss_host, float *grad_dev);
/* Network used by SEA_START_LEARNED (the state must outlive those calls). */
sea_status sea_nn_attach(sea_ctx *ctx, const void *state_dev);
/* Training samples from converged pair solves (the solve of
 * sea_exx_pair_solve with the context's options): for pair k,
 * x_dev[k*D^3..] = resample(rho/s) and t_dev[k*D^3..] = resample((v - v_ME)/s)
 * on D^3, s = dV sum |rho|; s_dev (nullable) receives s. */
sea_status sea_exx_nn_samples(sea_ctx *ctx, const sea_grid *grid, int n_occ, const void *phi_dev,
                              sea_dtype phi_dtype, int n_pairs, const sea_pair *pairs_host,
                              void *ws_dev, size_t ws_bytes, int D, float *x_dev, float *t_dev,
                              double *s_dev, sea_pair_stat *stats_host);

/* Milliseconds spent in each stage by the most recent profiled call that
 * ran it (HIP events on opts.hip_stream; waits for those events).  ms_out
 * holds SEA_STAGE_COUNT floats; stages not run by that call read 0. */
sea_status sea_stage_times(sea_ctx *ctx, float *ms_out);

/* Host evaluation of r^l Y_lm (real orthonormal, index l*l + l + m) at the
 * vector (x, y, z) by the same Cartesian recurrence the GPU kernels use;
 * out holds (lmax+1)^2 doubles.  lmax <= 6. */
sea_status sea_solid_harmonics_host(int lmax, double x, double y, double z, double *out);

#ifdef __cplusplus
}
#endif

#endif /* SEA_H */
