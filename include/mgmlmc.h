/*
 * mgmlmc.h -- C ABI of a single-GPU (MI355X, gfx950) library for multigrid
 * multilevel Monte Carlo trace estimation with orthogonal projectors
 * (Frommer, Jimenez-Merchan, Knechtli, Korzec, Ramirez-Hidalgo,
 * arXiv:2509.11424).
 *
 * The calls follow the paper's statement of the problem: build the level
 * hierarchy (Sec. 2.2: aggregation-based unitary P_l, Galerkin
 * D_{l+1} = P_l^H D_l P_l), draw Z4 probes (Sec. 1, eq. z4), and estimate a
 * trace, a connected correlator or disconnected loops per level with the
 * variance of every term (Sec. 3 decomposition; Sec. 4 variance estimator;
 * Sec. 4.1 correlator split; Sec. 4.3 loops).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Status codes are returned, never thrown; mgm_last_error() gives a
 *   thread-local message for the last failing call.
 * - Complex numbers are interleaved (re, im).
 * - Device pointers ("_dev") are plain device addresses (for example from
 *   torch tensors); host pointers ("_host") are ordinary host memory.  The
 *   library never frees memory it did not allocate.
 * - Device memory: the caller owns every device buffer, including the
 *   workspace handed to mgm_operator_create and mgm_hierarchy_create, whose
 *   size comes from the matching *_workspace_size call.  The workspace must
 *   stay valid and untouched until the object is destroyed.  The library
 *   itself allocates only small pinned host staging buffers.
 * - Lattice: dims = {X, Y, Z, T}; site s = x + X*(y + Y*(z + Z*t)).
 *   Fine dof per site d = 12, dof = 3*spin + colour, chiral gamma basis with
 *   gamma5 = diag(1, 1, -1, -1).  Level l >= 1 has d = 2*N_tv(l-1) dof per
 *   site, dof = N_tv*chi + k.
 * - Vector layout on every level ("dof-major"): a batch of nrhs vectors of a
 *   level with V_l sites and d_l dof per site is one array with element
 *   (dof, site, rhs) at index (dof*V_l + site)*nrhs + rhs.
 * - Gauge field input (host, FP64): [T][Z][Y][X][mu][3][3] complex,
 *   mu = 0..3 for x, y, z, t; U_mu(x) connects x + mu to x.
 * - All work is enqueued on the HIP stream given to mgm_context_create.
 *   Calls that return host results synchronise that stream.
 * - Handles are not thread safe; distinct contexts are independent.
 */
#ifndef MGMLMC_H
#define MGMLMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MGM_OK = 0,
  MGM_ERR_INVALID_ARG = -1,
  MGM_ERR_SHAPE = -2,
  MGM_ERR_WORKSPACE = -3,
  MGM_ERR_NOT_CONVERGED = -4,
  MGM_ERR_RANK_DEFICIENT = -5,
  MGM_ERR_NUMERIC = -6,
  MGM_ERR_HIP = -7
} mgm_status;

/* Storage precision of an operator application or a vector.
 * F64: double complex; F32: float complex; F16: IEEE half complex
 * (arithmetic in FP32); BF16 is used only for coarse-stencil MFMA operands. */
typedef enum { MGM_PREC_F64 = 0, MGM_PREC_F32 = 1, MGM_PREC_F16 = 2, MGM_PREC_BF16 = 3 } mgm_prec;

typedef struct mgm_context_s* mgm_context;
typedef struct mgm_operator_s* mgm_operator;
typedef struct mgm_hierarchy_s* mgm_hierarchy;

/* Human-readable name of a status code (static string). */
const char* mgm_status_string(mgm_status s);
/* Message describing the last error on this thread ("" if none). */
const char* mgm_last_error(void);
/* Library version string. */
const char* mgm_version(void);

/* ------------------------------------------------------------- context */

/* Binds the library to HIP device `device` and to `hip_stream` (a
 * hipStream_t, NULL for the default stream).  Every later call on this
 * context or on an object built from it makes that device current for its
 * duration and restores the caller's current device on return, so contexts
 * on different devices can be used from one thread.  Errors: INVALID_ARG, HIP. */
mgm_status mgm_context_create(int device, void* hip_stream, mgm_context* out);
/* Switches the stream used by later calls on this context. */
mgm_status mgm_context_set_stream(mgm_context ctx, void* hip_stream);
/* Launch-shape autotuner (project-written): when enabled, the first launch of
 * a tunable kernel (fine dslash: rhs per thread and block order of the
 * site-parallel kernel, then the tile, z-run and rhs group of the
 * plane-marching kernel; coarse stencils: 16-rhs tiles per workgroup) for a
 * given shape times every variant on that call's own arguments with HIP
 * events (best of three) and keeps the fastest for the rest of the context's
 * life.  Results do not depend on the variant beyond floating-point rounding
 * order.  Off by default (variant 0). */
mgm_status mgm_context_set_autotune(mgm_context ctx, int32_t enable);
/* Text table of the tuned shapes ("key variant ms_v0 ms_v1 ..." per line),
 * NUL-terminated, truncated to `bytes`; *needed receives the full length. */
mgm_status mgm_context_tune_report(mgm_context ctx, char* buf, size_t bytes, size_t* needed);
/* Pins launch variant `variant` (>= 0) for shape `key` (a key of the tune
 * report, e.g. from an earlier run), as if the autotuner had chosen it; later
 * launches of that shape use it whether or not tuning is enabled.  A variant
 * beyond the shape's count makes those launches fail with INVALID_ARG.
 * Errors: INVALID_ARG (NULL key, negative variant). */
mgm_status mgm_context_tune_set(mgm_context ctx, const char* key, int32_t variant);
void mgm_context_destroy(mgm_context ctx);

/* --------------------------------------------------------- fine operator */

/* The Wilson-clover Dirac operator (the paper requires only a discretised,
 * Gamma5-hermitian Dirac operator with 12 dof per site, Sec. 1 and Sec. 2.1):
 *   (D psi)(x) = (4 + m0) psi(x)
 *     - 1/2 sum_mu [(1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^H psi(x-mu)]
 *     + csw (i/4) sum_{mu != nu} sigma_mu_nu F_mu_nu(x) psi(x)
 * with clover-leaf F_mu_nu = (Q - Q^H)/8 and, if t_antiperiodic != 0, a
 * factor -1 on hops across the time boundary. */
typedef struct {
  int32_t dims[4];        /* X, Y, Z, T; each >= 2 */
  double m0;              /* bare mass */
  double csw;             /* clover coefficient (0: plain Wilson) */
  int32_t t_antiperiodic; /* 1: antiperiodic in time, 0: periodic */
} mgm_lattice_desc;

/* Workspace (bytes) needed by mgm_operator_create: links and clover blocks
 * in FP64, FP32 and FP16.  Errors: INVALID_ARG, SHAPE. */
mgm_status mgm_operator_workspace_size(const mgm_lattice_desc* desc, size_t* bytes);

/* Copies the FP64 gauge field from host memory (layout above), builds the
 * clover term on the GPU and keeps FP32/FP16 copies.  `ws_dev` must hold
 * mgm_operator_workspace_size bytes, 256-byte aligned.
 * Errors: INVALID_ARG, SHAPE, WORKSPACE, HIP. */
mgm_status mgm_operator_create(mgm_context ctx, const mgm_lattice_desc* desc,
                               const double* gauge_host, void* ws_dev, size_t ws_bytes,
                               mgm_operator* out);

/* y = D x for nrhs vectors in dof-major layout, in precision `prec`
 * (F64, F32 or F16; x and y hold elements of that precision).  x and y must
 * not overlap.  Errors: INVALID_ARG, HIP. */
mgm_status mgm_operator_apply(mgm_operator op, mgm_prec prec, const void* x_dev, void* y_dev,
                              int32_t nrhs);

/* Scratch bytes needed by mgm_operator_apply_dot for (prec, nrhs). */
mgm_status mgm_operator_dot_workspace_size(mgm_operator op, mgm_prec prec, int32_t nrhs, size_t* bytes);

/* y = D x as mgm_operator_apply, fused with the two reductions of a
 * minimal-residual step: yx_dev[r] = y_r^H x_r (complex, FP64) and
 * yy_dev[r] = |y_r|^2 (FP64) per right-hand side, summed in a fixed order from
 * the stored (rounded) y.  ws_dev: caller-owned device scratch of
 * mgm_operator_dot_workspace_size bytes, 256-byte aligned.  nrhs <= 256.
 * Errors: INVALID_ARG, WORKSPACE, HIP. */
mgm_status mgm_operator_apply_dot(mgm_operator op, mgm_prec prec, const void* x_dev, void* y_dev,
                                  int32_t nrhs, void* ws_dev, size_t ws_bytes, void* yx_dev,
                                  void* yy_dev);

/* Allocation-free form of mgm_operator_apply_dot, for callers that cannot
 * allocate device memory or hand over a workspace (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments and results as mgm_operator_apply_dot without ws_dev / ws_bytes:
 * the reduction partials live in one fixed device array of the library,
 * MGM_NOALLOC_SCRATCH_BYTES per GPU, held from the first mgm_context_create
 * on that GPU until the process ends.  A call needs
 * mgm_operator_dot_workspace_size(op, prec, nrhs) <= MGM_NOALLOC_SCRATCH_BYTES
 * (for example up to 32 rhs on a 16^4 lattice, up to 4 on 32^3 x 64);
 * larger shapes return MGM_ERR_WORKSPACE without launching anything.  The
 * call allocates no device or host memory.  Every call on one GPU shares the
 * array: calls that overlap on one GPU (other streams, other threads) race;
 * calls ordered on one stream do not.  Nothing in the array needs clearing
 * (each call writes every partial it reads).
 * Errors: INVALID_ARG, WORKSPACE, HIP. */
#define MGM_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
mgm_status mgm_operator_apply_dot_noalloc(mgm_operator op, mgm_prec prec, const void* x_dev, void* y_dev,
                                          int32_t nrhs, void* yx_dev, void* yy_dev);

/* One fused step of the FP16 minimal-residual smoother with the previous
 * step's length (the minimal-residual smoother of this library's multigrid
 * solver as a Richardson step of lagged MR length; the paper fixes only that
 * the levels are solved by multigrid, Sec. 4, so this smoother is a reading
 * of this library, not a passage of the paper): with
 * omega_r = qr_prev_dev[r] / qq_prev_dev[r] (0 where qq_prev_dev[r] is 0) and
 * q = D r (not stored), writes r_next = r - omega q, updates x += omega r in
 * place, and yx_dev[r] = q_r^H r_r, yy_dev[r] = |q_r|^2 (FP64 sums of the
 * FP32 q), which give the next step's length.  r, r_next and x
 * are distinct FP16 dof-major (12, V, nrhs) complex-pair arrays; qr_prev /
 * qq_prev may coincide with yx / yy (they are read first).  Workspace as
 * mgm_operator_apply_dot with prec F16.  Errors: INVALID_ARG; SHAPE when no
 * plane-marching tile fits the lattice and nrhs (mgm_operator_step_fusable);
 * WORKSPACE; HIP. */
mgm_status mgm_operator_smoother_step(mgm_operator op, const void* r_dev, void* r_next_dev, void* x_dev,
                                      const void* qr_prev_dev, const void* qq_prev_dev, int32_t nrhs,
                                      void* ws_dev, size_t ws_bytes, void* yx_dev, void* yy_dev);
/* 1 when mgm_operator_smoother_step runs for this rhs count, else 0. */
int32_t mgm_operator_step_fusable(mgm_operator op, int32_t nrhs);

/* Number of lattice sites of the fine operator. */
int64_t mgm_operator_sites(mgm_operator op);
void mgm_operator_destroy(mgm_operator op);

/* ----------------------------------------------------------------- probes */

/* Z4 probe entries (eq. z4): entry i of probe p is
 * (1, i, -1, -i)[w0 >> 30] with w0 the first output word of Philox4x32-10
 * (Salmon et al., SC'11) at key (seed & 0xffffffff, seed >> 32) and counter
 * (i & 0xffffffff, i >> 32, p, stream).  `stream` = 256*level + kind with
 * kind 0 plain, 1 O_l, 2 F_l, 3 M_l, 4 coarsest, 5 correlator source,
 * 6 loop source, 7 test vector, 8 network training input.  Writes nprobe vectors of n_site*dof entries
 * in dof-major layout (probe p = first_probe + rhs; entry index
 * i = site*dof + dof_index) to out_dev in precision `prec` (F64 or F32).
 * Errors: INVALID_ARG, HIP. */
mgm_status mgm_draw_z4(mgm_context ctx, uint64_t seed, uint32_t stream, uint64_t first_probe,
                       int32_t nprobe, int64_t n_site, int32_t dof, mgm_prec prec,
                       void* out_dev);

/* Probe distributions (Sec. 1: entries i.i.d. with E[x] = 0 and
 * E[conj(x_i) x_j] = delta_ij; Z4 is eq. z4, the others are the alternatives
 * named after eq. variance-Frobenius-Relation), all from the Philox4x32-10
 * words w of the entry's counter as in mgm_draw_z4:
 *   Z4: (1, i, -1, -i)[w0 >> 30]        Z2: 1 - 2 (w0 >> 31)
 *   U1: exp(2 pi i (w0 + 1/2) 2^-32)    (uniform on the unit circle)
 *   GAUSS: real standard normal by the Box-Muller transform of
 *          u1 = (w0 + 1) 2^-32, u2 = w1 2^-32: sqrt(-2 ln u1) cos(2 pi u2). */
typedef enum { MGM_NOISE_Z4 = 0, MGM_NOISE_Z2 = 1, MGM_NOISE_U1 = 2, MGM_NOISE_GAUSS = 3 } mgm_noise_kind;

/* mgm_draw_z4 for any distribution of mgm_noise_kind (Z4 and Z2 bit-exact
 * functions of the counter; U1 and GAUSS through FP64 cos / sin / log / sqrt).
 * Errors: INVALID_ARG, HIP. */
mgm_status mgm_draw_noise(mgm_context ctx, int32_t kind, uint64_t seed, uint32_t stream, uint64_t first_probe,
                          int32_t nprobe, int64_t n_site, int32_t dof, mgm_prec prec, void* out_dev);

/* -------------------------------------------------------------- hierarchy */

#define MGM_MAX_LEVELS 4

/* Multigrid hierarchy (Sec. 2.2).  Level l >= 1 is the Galerkin operator of
 * level l-1 on aggregates of block[l-1] sites, built from ntv[l-1] test
 * vectors (Z4 starts, setup_steps rounds of setup_mr minimal-residual steps
 * on D_{l-1}, normalised) orthonormalised per (aggregate, chirality) block by
 * modified Gram-Schmidt with re-orthogonalisation (diag R > 0). */
typedef struct {
  int32_t nlevels;                    /* 2..MGM_MAX_LEVELS */
  int32_t block[MGM_MAX_LEVELS - 1][4];
  int32_t ntv[MGM_MAX_LEVELS - 1];    /* test vectors per transfer, 1..128 (coarse dof 2 ntv) */
  int32_t setup_steps;                /* default 20 */
  int32_t setup_mr;                   /* default 4 */
  uint64_t seed;                      /* test-vector probes (kind 7) */
  int32_t max_nrhs;                   /* largest batch of right-hand sides */
  int32_t restart;                    /* FGMRES restart length, >= 2 */
  int32_t mixed;                      /* 0: FP64 solver workspaces only;
                                         1: FP32 Krylov workspaces plus FP32/BF16
                                         copies of P and D_c for the mixed solver
                                         (FP64 keeps only defect-correction vectors);
                                         2: both full */
  int32_t with_corr;                  /* 1: reserve the fine-level term vectors needed
                                         by CORR_PS and LOOPS estimates */
  int32_t max_nrhs_level[MGM_MAX_LEVELS]; /* optional per-level batch capacity (0: max_nrhs);
                                         level l holds max over levels <= l, so
                                         coarse levels can batch more right-hand
                                         sides than the fine level */
} mgm_hierarchy_desc;

mgm_status mgm_hierarchy_workspace_size(mgm_operator op, const mgm_hierarchy_desc* desc,
                                        size_t* bytes);

/* Builds the hierarchy on the GPU.  Errors: INVALID_ARG, SHAPE, WORKSPACE,
 * RANK_DEFICIENT (a test-vector block lost rank), NUMERIC, HIP. */
mgm_status mgm_hierarchy_create(mgm_operator op, const mgm_hierarchy_desc* desc, void* ws_dev,
                                size_t ws_bytes, mgm_hierarchy* out);

/* Dimension bookkeeping of level `level`: sites, dof per site, n = sites*dof. */
mgm_status mgm_hierarchy_level_info(mgm_hierarchy h, int32_t level, int64_t* sites,
                                    int32_t* dof, int64_t* n);

/* What mgm_hierarchy_export copies to host memory. */
typedef enum {
  MGM_EXPORT_AGG_MAP = 0,  /* int64 [Vc][2][rows]: flat dof index (site*d + chi*d/2 + j)
                              of block row loc*(d/2) + j of aggregate a, chirality chi */
  MGM_EXPORT_P = 1,        /* complex FP64 [Vc][2][rows][ntv] */
  MGM_EXPORT_COARSE = 2,   /* complex FP64 [Vc][9][dc][dc] stencil of D_{level+1};
                              dir 0 self, 1+mu forward, 5+mu backward */
  MGM_EXPORT_TV = 3        /* complex FP64 [ntv][n_level] test vectors (before QR) */
} mgm_export_kind;

/* Copies one object of transfer `level` (0 <= level < nlevels-1) to
 * host_buf, which must hold `bytes` >= the object size.  Synchronises. */
mgm_status mgm_hierarchy_export(mgm_hierarchy h, int32_t level, mgm_export_kind what,
                                void* host_buf, size_t bytes);

/* Level operators applied in FP64 (fine: the Wilson-clover stencil; coarse:
 * the nine-point Galerkin stencil), and the transfers:
 *   restrict: y_c = P_l^H x, prolong: y = P_l x_c, project: y = (I - P_l P_l^H) x
 * all in dof-major FP64 layout. */
mgm_status mgm_level_apply(mgm_hierarchy h, int32_t level, const void* x_dev, void* y_dev,
                           int32_t nrhs);
/* The same in precision `prec`: F64 (double complex vectors), F32 (float
 * complex vectors, FP32 operator), F16 (level 0 only, half complex vectors),
 * BF16 (level >= 1; float complex vectors, operator and vectors rounded to
 * BF16 for the matrix cores, FP32 accumulation).  F32 and BF16 coarse
 * operators exist only in hierarchies built with mixed != 0. */
mgm_status mgm_level_apply_prec(mgm_hierarchy h, int32_t level, mgm_prec prec, const void* x_dev,
                                void* y_dev, int32_t nrhs);
mgm_status mgm_restrict(mgm_hierarchy h, int32_t level, const void* x_dev, void* y_dev,
                        int32_t nrhs);
mgm_status mgm_prolong(mgm_hierarchy h, int32_t level, const void* x_dev, void* y_dev,
                       int32_t nrhs);
mgm_status mgm_project_out(mgm_hierarchy h, int32_t level, const void* x_dev, void* y_dev,
                           int32_t nrhs);
/* Restriction and prolongation (Sec. 2.2: y_c = P_l^H x, y = P_l x_c) in
 * precision `prec`: F64 as mgm_restrict / mgm_prolong, or F32 (float complex
 * dof-major vectors, P_l stored in FP16, FP32 arithmetic; the transfers of
 * the mixed V-cycle, present only in hierarchies built with mixed != 0).
 * Other precisions return MGM_ERR_INVALID_ARG. */
mgm_status mgm_restrict_prec(mgm_hierarchy h, int32_t level, mgm_prec prec, const void* x_dev,
                             void* y_dev, int32_t nrhs);
mgm_status mgm_prolong_prec(mgm_hierarchy h, int32_t level, mgm_prec prec, const void* x_dev,
                            void* y_dev, int32_t nrhs);
/* The transfers of the mixed V-cycle whose fine-side vector is stored in FP16
 * (half complex, dof-major) and scaled per right-hand side by scale_dev
 * (device, nrhs doubles), with FP16-stored P_l and FP32 arithmetic (Sec. 2.2):
 *   mgm_restrict_f16:    y_c = P_l^H (scale x16)          (y_c float complex)
 *   mgm_prolong_add_f16: y = scale x16 + P_l x_c          (x_c, y float complex)
 * Hierarchies built with mixed != 0 only; y and the inputs must not overlap. */
mgm_status mgm_restrict_f16(mgm_hierarchy h, int32_t level, const void* x16_dev, const double* scale_dev,
                            void* y_dev, int32_t nrhs);
mgm_status mgm_prolong_add_f16(mgm_hierarchy h, int32_t level, const void* xc_dev, const void* x16_dev,
                               const double* scale_dev, void* y_dev, int32_t nrhs);

/* ------------------------------------------------------------------ solve */

typedef enum {
  MGM_SOLVE_MG = 0,        /* FP64 FGMRES preconditioned by an FP64 MG V-cycle */
  MGM_SOLVE_MG_MIXED = 1,  /* FP64 defect correction around FP32 FGMRES with a
                              V-cycle of FP16-storage fine smoothing, FP16 P and
                              BF16-MFMA coarse operators */
  MGM_SOLVE_GMRES = 2,     /* unpreconditioned FP64 GMRES */
  MGM_SOLVE_NET = 3        /* MG_MIXED with the learned smoother (mgm_net) */
} mgm_solve_kind;

typedef struct {
  double tol;          /* stop when every |b - D x| / |b| <= tol (true FP64 residual) */
  int32_t maxiter;     /* outer iteration cap */
  int32_t kind;        /* mgm_solve_kind */
  int32_t smooth;      /* minimal-residual smoothing steps (pre and post) on the
                          fine level (level 0) */
  int32_t coarse_iters;/* iterations of the coarse-level solve inside a V-cycle */
  double inner_tol;    /* MG_MIXED: relative reduction per FP32 inner solve */
  void* net;           /* MGM_SOLVE_NET: network handle (mgm_net), else NULL */
  int32_t coarse_bf16; /* MG_MIXED / NET: coarse-level operators inside the V-cycle
                          use BF16 MFMA operands with FP32 accumulation (1) or
                          FP32 (0); the Arnoldi operator of every solve stays FP32 */
  int32_t smoother_f16;/* MG_MIXED / NET: the fine-level MR smoother stores its
                          vectors in FP16 (1; inputs scaled per rhs to unit RMS
                          entries, FP32 arithmetic) or FP32 (0) */
  int32_t smooth_coarse; /* MR smoothing steps on levels >= 1 (0: the same as smooth) */
  int32_t graphs;      /* 1: the coarse-grid correction below each level (a fixed
                          launch sequence per level, precision and batch) is
                          captured into a HIP graph on its second use and
                          replayed afterwards; needs a non-NULL context stream
                          (ignored otherwise).  Results are identical to 0. */
} mgm_solve_desc;

typedef struct {
  int32_t iterations;  /* total outer Arnoldi steps (all right-hand sides together) */
  int32_t restarts;    /* FGMRES cycles */
  int32_t fallbacks;   /* NET: cycles that fell back to plain MG */
  double max_rel_residual;  /* largest final true relative residual */
  double seconds;      /* wall time of the call */
} mgm_solve_stats;

/* Solves D_level x = b for nrhs right-hand sides (dof-major FP64), x0 = 0.
 * Every right-hand side is judged by its own true FP64 residual.  Returns
 * NOT_CONVERGED (with x and stats written) if any misses tol within maxiter. */
mgm_status mgm_solve(mgm_hierarchy h, int32_t level, const mgm_solve_desc* desc,
                     const void* b_dev, void* x_dev, int32_t nrhs, mgm_solve_stats* stats);

/* ------------------------------------------------- hierarchy refinement */

/* More accurate fine test vectors (Sec. 5: test vectors computed to smaller
 * eigen-residuals strengthen the coarse space).  Starting from the rough
 * vectors of the hierarchy's recipe (orthonormalised), alternates a
 * Rayleigh-Ritz step on the Hermitian Q = Gamma5 D over span(V) (Ritz pairs
 * ordered by |theta| ascending, each vector's phase fixed so that the sum of
 * its entries is real and positive) with inverse block power steps
 * V <- QR(D^-1 Gamma5 V) (solves with `solve` at tolerance power_tol, batch
 * columns at a time), until every Ritz pair has the eigen-residual
 * rho = |Q v - theta v| / |theta| <= eig_tol or max_iters steps are done.  The
 * Ritz vectors then replace the test vectors of transfer 0: P_0, D_1 and every
 * coarser level (rough recipe) are rebuilt in place.  N_tv stays ntv[0]. */
typedef struct {
  int32_t max_iters;    /* inverse block power steps, at most */
  double eig_tol;       /* target eigen-residual of every Ritz pair (the paper: 1e-4) */
  double power_tol;     /* relative residual of the power-step solves */
  int32_t batch;        /* columns per solver launch, 1..fine-level capacity */
  mgm_solve_desc solve; /* solver of the power steps (tolerance replaced by power_tol) */
} mgm_refine_desc;

typedef struct {
  int32_t steps;         /* power steps taken */
  int32_t converged;     /* 1 if every power-step solve reached power_tol */
  double max_rho_start;  /* largest eigen-residual of the rough vectors */
  double max_rho;        /* largest eigen-residual of the final vectors */
  double seconds;        /* wall time including the rebuild */
} mgm_refine_stats;

/* Device bytes of the refinement's temporary workspace (three blocks of
 * ntv[0] fine vectors, FP64). */
mgm_status mgm_hierarchy_refine_workspace_size(mgm_hierarchy h, size_t* bytes);
/* Runs the refinement in the caller's temporary workspace (free afterwards).
 * rho_host / theta_host (host, ntv[0] doubles each, may be NULL) receive the
 * final eigen-residuals and Ritz values.  Errors: INVALID_ARG, WORKSPACE,
 * RANK_DEFICIENT, NUMERIC, HIP. */
mgm_status mgm_hierarchy_refine(mgm_hierarchy h, const mgm_refine_desc* desc, void* ws_dev, size_t ws_bytes,
                                mgm_refine_stats* stats, double* rho_host, double* theta_host);

/* ------------------------------------------------ learned preconditioner */

/*
 * Gauge-covariant parallel-transport convolution (PTC) network used as the
 * fine-level smoother of the multigrid preconditioner (solve kind NET).  The
 * paper does not describe a learned preconditioner: this is the learned form
 * of the hot path.  One layer maps c_in to c_out colour-triplet channels,
 *
 *   out_a(x) = sum_p sum_b W_p[a][b] (T_p in_b)(x),
 *
 * over nine paths p: 0 identity, 1 + mu forward transport U_mu(x) in(x + mu),
 * 5 + mu backward transport U_mu(x - mu)^H in(x - mu) (mu = x, y, z, t; the
 * antiperiodic time sign as in the Dirac operator).  Input and output are
 * fine spinors (4 spin channels); layers are linear.  Inside the V-cycle the
 * network replaces the fine smoother: M r = e_c + N(r - D e_c) with
 * e_c = P D_c^-1 P^H r.  Vectors are FP32 complex, dof-major
 * [(channel * 3 + colour)][site][rhs] (a spinor is channels 0..3).
 *
 * Weights: complex, interleaved, ordered [layer][path][c_out][c_in]; the
 * gradient of a real loss L with respect to a complex weight w is reported as
 * dL/dRe(w) + i dL/dIm(w).  The network keeps FP64 master weights and Adam
 * state; kernels use an FP32 copy.
 */
#define MGM_NET_MAX_LAYERS 8

typedef struct mgm_net_s* mgm_net;

typedef struct {
  int32_t nlayers;                          /* 1..MGM_NET_MAX_LAYERS */
  int32_t width[MGM_NET_MAX_LAYERS + 1];    /* channels; width[0] = width[nlayers] = 4,
                                               every width in {4, 8, 12, 16} */
  uint64_t seed;                            /* initial weights (identity path plus small noise) */
  int32_t max_nrhs;                         /* right-hand sides per application, 1..256 */
  int32_t train_nrhs;                       /* training pairs (= batch), 0..256; 0: no training */
  int32_t bf16_weights;                     /* 1: the layers use the weights rounded to BF16
                                               (nearest, ties to even) with FP32 accumulation;
                                               the FP64 master weights and Adam stay unrounded
                                               and the gradient is taken at the rounded weights */
} mgm_net_desc;

typedef struct {
  int32_t steps;       /* Adam steps (full batch) */
  double lr;           /* learning rate */
  double beta1, beta2, eps;  /* Adam constants (0: 0.9, 0.999, 1e-8) */
  uint64_t seed;       /* Z4 draws of the training inputs */
  double target_tol;   /* FP64 solves that make the training targets */
} mgm_train_desc;

typedef struct {
  double loss_first;   /* loss at the initial weights */
  double loss_last;    /* loss at the weights before the last update */
  int32_t steps;
  double seconds;      /* wall time including target generation */
} mgm_train_stats;

/* Device bytes of the network's workspace on operator op's lattice. */
mgm_status mgm_net_workspace_size(mgm_operator op, const mgm_net_desc* desc, size_t* bytes);
/* Creates the network in the caller's workspace (256-byte aligned device
 * memory of at least the queried size, owned by the caller and kept until
 * mgm_net_destroy).  op must outlive the network.  Bad widths or counts:
 * MGM_ERR_INVALID_ARG; small workspace: MGM_ERR_WORKSPACE. */
mgm_status mgm_net_create(mgm_operator op, const mgm_net_desc* desc, void* ws_dev, size_t ws_bytes,
                          mgm_net* out);
/* Moves the network to another operator of the same lattice (another gauge
 * field): later applications and training use that operator's links; the
 * weights and the Adam state are kept (the layers are gauge covariant, their
 * weights do not depend on the field).  Errors: INVALID_ARG, SHAPE. */
mgm_status mgm_net_bind(mgm_net net, mgm_operator op);
mgm_status mgm_net_num_weights(mgm_net net, int64_t* count);  /* complex weights */
/* Host FP64 weights (2 * count doubles); set also resets the Adam state. */
mgm_status mgm_net_set_weights(mgm_net net, const double* w_host);
mgm_status mgm_net_get_weights(mgm_net net, double* w_host);
/* Writes the network's layer count, widths and FP64 master weights to the
 * file `path` (a small binary file: the 8 bytes "MGMNET01", int32 nlayers,
 * int32 width[9], int64 count, then 2 * count little-endian doubles).
 * Errors: INVALID_ARG (NULL), HIP, NUMERIC (the file cannot be written). */
mgm_status mgm_net_save(mgm_net net, const char* path);
/* Reads such a file into the network (as mgm_net_set_weights, resetting the
 * Adam state).  A file for other layers or widths: MGM_ERR_SHAPE; a missing,
 * short or foreign file: MGM_ERR_INVALID_ARG. */
mgm_status mgm_net_load(mgm_net net, const char* path);
/* y = N(r) for nrhs <= max_nrhs fine spinors (FP32 complex, device). */
mgm_status mgm_net_apply(mgm_net net, const void* r_dev, void* y_dev, int32_t nrhs);
/* Loss (1/nrhs) sum_j |N(r_j) - e_j|^2 / |e_j|^2 and its weight gradient
 * (host, 2 * count doubles, same order as the weights) for nrhs <= train_nrhs
 * pairs.  Needs train_nrhs > 0. */
mgm_status mgm_net_loss_grad(mgm_net net, const void* r_dev, const void* e_dev, int32_t nrhs, double* loss,
                             double* grad_host);
/* Trains with full-batch Adam on train_nrhs pairs (r, e): r is the fine
 * residual left by the coarse-grid correction of a Z4 vector
 * (r = z - D P D_c^-1 P^H z) and e = D^-1 r from FP64 MG solves of hierarchy
 * h, which must be built on the network's operator with max_nrhs >= train_nrhs
 * on levels 0 and 1.  loss_history (host, steps doubles) may be NULL. */
mgm_status mgm_net_train(mgm_net net, mgm_hierarchy h, const mgm_train_desc* desc, mgm_train_stats* stats,
                         double* loss_history);
void mgm_net_destroy(mgm_net net);

/* --------------------------------------------------------------- estimate */

typedef enum { MGM_OBS_TRACE = 0, MGM_OBS_CORR_PS = 1, MGM_OBS_LOOPS = 2 } mgm_observable;
typedef enum { MGM_DEC_PLAIN = 0, MGM_DEC_OBLIQUE = 1, MGM_DEC_ORTHOGONAL = 2, MGM_DEC_DEFLATED = 3 } mgm_decomposition;

/*
 * Term numbering (L = nlevels):
 *  TRACE  plain:      [0] x^H D^-1 x
 *         oblique:    [l] M_l (l < L-1), [L-1] coarsest
 *         orthogonal: [l] O_l, [L-1+l] F_l (l < L-1), [2L-2] coarsest
 *  CORR_PS / LOOPS: terms B_r of the paper's correlator split (Sec. 4.1),
 *         plain [0] D^-1; oblique [l] B_l (l <= L-1); orthogonal
 *         [l] J_l, [L-1+l] K_l, [2L-2] coarsest.  Correlator results are
 *         per pair (r, s) in row-major order r*R + s.
 *  TRACE  deflated (Sec. 2.1, eq. deflated-estimator; needs `deflation`):
 *         [0] x^H (I - V V^H) D^-1 x with nprobe[0] Z4 probes (stream kind 10),
 *         [1] tr(V^H D^-1 V), computed once when the basis was built: one
 *         sample, variance 0, cost_s = the seconds of its k solves.
 * Probe groups: nprobe[g] probes for every term (TRACE, LOOPS) or pair
 * (CORR_PS) whose finest level is g; plain uses nprobe[0].
 */
typedef struct mgm_deflation_s* mgm_deflation;
typedef struct {
  int32_t observable;       /* mgm_observable */
  int32_t decomposition;    /* mgm_decomposition */
  int32_t nprobe[MGM_MAX_LEVELS];
  uint64_t seed;
  uint64_t first_probe;     /* probe index offset (restart / sharding) */
  int32_t batch;            /* right-hand sides per solver launch (<= max_nrhs) */
  mgm_solve_desc solve;
  int32_t batch_level[MGM_MAX_LEVELS]; /* optional batch per probe group g (0: batch);
                                          must not exceed the capacity of level g */
  mgm_deflation deflation;  /* MGM_DEC_DEFLATED: a basis built on this hierarchy, else NULL */
  int32_t noise;            /* probe distribution (mgm_noise_kind; 0 = Z4) of every term */
  int32_t probing;          /* LOOPS: probing distance p >= 1 (0 or 1: none).  Every source is
                               split into the p^4 colours of the block pattern
                               colour(x) = (x mod p) + p((y mod p) + p((z mod p) + p(t mod p)))
                               (p must divide every fine extent); a probe's value is the
                               sum over colours of the coloured sources' values, one
                               application of every term per colour (Sec. 5: probing
                               combined with the multilevel decomposition) */
} mgm_estimate_desc;

typedef struct {
  int32_t nterms;           /* TRACE, LOOPS: terms; CORR_PS: pairs R*R */
  int32_t T;                /* time extent (1 for TRACE) */
  int32_t ngamma;           /* 6 for LOOPS, else 1 */
  int64_t nsamples;         /* entries of `samples` */
} mgm_estimate_sizes;

/* Caller-owned host arrays (sizes from mgm_estimate_sizes).  Per term (and
 * per t, Gamma): N, mean (complex), variance sum|X - mean|^2/(N-1) (Sec. 4);
 * cost_s = solver seconds spent per sample.  `samples` (optional, may be
 * NULL) receives every per-probe complex value ordered
 * [term][probe][gamma][t].  total_mean / total_var: sum over terms of the
 * means and of var/N (independent probe sets); per t for CORR_PS / LOOPS. */
typedef struct {
  int64_t* n;               /* [nterms] */
  double* mean;             /* [nterms][ngamma][T] complex */
  double* var;              /* [nterms][ngamma][T] */
  double* cost_s;           /* [nterms] */
  double* samples;          /* [nsamples] complex, or NULL */
  double* total_mean;       /* [ngamma][T] complex */
  double* total_var;        /* [ngamma][T] */
  mgm_solve_stats stats;    /* accumulated over all solves */
} mgm_estimate_result;

mgm_status mgm_estimate_sizes_query(mgm_hierarchy h, const mgm_estimate_desc* desc,
                                    mgm_estimate_sizes* sizes);
mgm_status mgm_estimate(mgm_hierarchy h, const mgm_estimate_desc* desc, mgm_estimate_result* out);

/* -------------------------------------------------------------- deflation */

/* Inexact deflation basis of the fine operator (Sec. 2.1, "Deflation for the
 * Dirac operator"; setup of Sec. 4.2): V (n x k, orthonormal columns)
 * approximates the eigenvectors of the Hermitian Gamma5 D belonging to its
 * smallest |eigenvalues|.  Start: k Z4 columns (stream kind 9 of level 0,
 * probe index = column), orthonormalised; then power_iters inverse block
 * power steps V <- QR(D^-1 Gamma5 V), the solves to power_tol.  QR: the
 * unique factor with positive real diag(R) (CholeskyQR applied twice; a
 * column whose component outside the earlier ones falls below 1e-12 of its
 * norm: MGM_ERR_RANK_DEFICIENT).  After the power steps the exact term
 * tr(V^H D^-1 V) is computed with `solve` (its tolerance).  Solves run in
 * batches of `batch` columns on the hierarchy's fine level. */
typedef struct {
  int32_t k;            /* basis columns, 1..1024 */
  int32_t power_iters;  /* inverse block power steps (the paper: 5) */
  double power_tol;     /* relative residual of the power-step solves (the paper: 1e-6) */
  uint64_t seed;        /* start block */
  int32_t batch;        /* columns per solver launch, 1..fine-level capacity */
  mgm_solve_desc solve; /* solver of the power steps (tolerance replaced by power_tol)
                           and of the exact term */
} mgm_deflation_desc;

/* Device bytes of the basis workspace: V (n x k complex FP64) plus the
 * partial sums of its tall-skinny products. */
mgm_status mgm_deflation_workspace_size(mgm_hierarchy h, const mgm_deflation_desc* desc, size_t* bytes);
/* Builds the basis in the caller's workspace (256-byte aligned, kept until
 * mgm_deflation_destroy; h must outlive it).  Errors: INVALID_ARG,
 * WORKSPACE, RANK_DEFICIENT, NOT_CONVERGED (a solve missed its tolerance; the
 * basis is still returned), NUMERIC, HIP. */
mgm_status mgm_deflation_create(mgm_hierarchy h, const mgm_deflation_desc* desc, void* ws_dev, size_t ws_bytes,
                                mgm_deflation* out);
/* Copies V to host memory as one dof-major block of k vectors: element
 * (dof, site, column) at (dof * V + site) * k + column, complex FP64;
 * host_buf must hold n * k * 16 bytes.  Synchronises. */
mgm_status mgm_deflation_export(mgm_deflation f, double* host_buf, size_t bytes);
/* tr(V^H D^-1 V) (complex, 2 doubles), and the seconds of the basis setup and
 * of the exact term. */
mgm_status mgm_deflation_info(mgm_deflation f, double* exact_trace, double* setup_s, double* exact_s);
void mgm_deflation_destroy(mgm_deflation f);

/* ------------------------------------------------------------------- MLMC */

/* Optimal sample sizes for target variance eps2 (Sec. 2.2, eq. MLMC-Nl):
 * N_l = ceil(eps2^-1 sqrt(V_l/C_l) sum_i sqrt(V_i C_i)), at least 2.
 * Pure host function.  Errors: INVALID_ARG. */
mgm_status mgm_mlmc_allocate(int32_t nterms, const double* var, const double* cost, double eps2,
                             int64_t* n_out);

/* -------------------------------------------------------------- profiling */

/* Kernel-level event timing of the library's own launches (dslash, coarse
 * stencil, transfers), off by default.  mgm_profile_query returns the number
 * of launches, their summed duration in ms and the summed algorithmic bytes
 * of kernel class `kclass` (0 fine dslash F64, 1 F32, 2 F16, 3 coarse stencil
 * F64, 4 coarse stencil F32, 5 coarse stencil BF16 MFMA, 6 restrict/prolong,
 * 7 network layers, 8 fused FP16 smoother steps).
 * Synchronises. */
mgm_status mgm_profile_enable(mgm_context ctx, int32_t on);
mgm_status mgm_profile_reset(mgm_context ctx);
mgm_status mgm_profile_query(mgm_context ctx, int32_t kclass, int64_t* launches, double* ms,
                             double* bytes);

void mgm_hierarchy_destroy(mgm_hierarchy h);

#ifdef __cplusplus
}
#endif
#endif /* MGMLMC_H */
