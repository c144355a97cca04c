/*
 * amgdd.h -- C ABI of the MI355X AMG-DD solve-phase library.
 *
 * Method: Mitchell, Strzodka, Falgout, "Parallel Performance of Algebraic
 * Multigrid Domain Decomposition (AMG-DD)".
 *   - AMG hierarchy (Section 2): classical Ruge-Stueben first-pass coarsening,
 *     direct interpolation, R = P^T, Galerkin A_{l+1} = R A P, down to a
 *     small coarsest level solved directly.
 *   - Composite grids (Section 3, Figure 1): per subdomain, padding eta_l
 *     through the graph of A_l on every level, C-points carried down, the
 *     coarsest level stored whole; ghost layer Dbar_l (Section 4.1).
 *   - AlgFAC cycle (Algorithm 4, Section 4.5) on every composite grid.
 *   - AMG-DD outer iteration (Algorithm 2): fine residual, restriction to all
 *     levels, composite right-hand sides, local AlgFAC, correction patched on
 *     each owned subdomain.
 *   - AMG V(1,1) cycle (Algorithm 1) on the same hierarchy.
 *   - Hybrid AMG-DD V(1,1) cycle (Algorithm 3, Section 3.1): V-cycle on the
 *     levels above a transition level, one AMG-DD cycle on the transition
 *     level's problem as the coarse solver (amgdd_params.hybrid_level).
 * The linear system is given by its fine-grid matrix alone, as the paper
 * states the problem (Section 2), plus a partition into subdomains
 * (Section 3) and the padding / number of AlgFAC cycles (Section 6.1).
 *
 * Relaxation is point l1-Jacobi: u <- u + (f - A u) / d, d_i = sum_j |a_ij|.
 *
 * Conventions for every entry point:
 *   - Host arrays are borrowed for the duration of the call and copied.
 *   - Device pointers (suffix _dev) are caller-owned HIP device memory on the
 *     handle's device (for example torch tensor storage); they must stay valid
 *     until the call returns.  All device work is enqueued on the handle's
 *     stream; the solve calls synchronise that stream once per outer iteration
 *     to read the residual norms, and return with the stream drained.
 *   - Nothing aborts.  Every call returns a status; amgdd_last_error() gives a
 *     thread-local message for the last non-OK status.
 *   - A handle is used by one host thread at a time.
 *   - Batched handles (amgdd_setup_composite_batch) see device vectors as the
 *     concatenation of the problems' vectors in setup order.
 *
 * Environment variables read when a handle is created (measurement and
 * testing; none changes the method):
 *   AMGDD_TRACE=1         roctx ranges around setup, upload, autotuning,
 *                         capture, solves and iterations (the roctx library
 *                         is opened with dlopen only then)
 *   AMGDD_THREADS=n       host threads of the setup (default: all)
 *   AMGDD_INDEX32         int32 column indices everywhere
 *   AMGDD_UNPAIRED        one entry per lane and load step everywhere
 *   AMGDD_QUAD            four entries per lane and load step everywhere
 *   AMGDD_SORT_WINDOW=n   row-sorting window on grouped levels (default 512;
 *                         0: local order)
 *   AMGDD_LANE_TARGET=x   entries per lane that set the lanes per composite row
 *   AMGDD_SERIAL          one stream per iteration (no side-stream branch)
 *   AMGDD_TEST_MAX_BYTES=n  device-memory cap (failure-path tests)
 *   AMGDD_WG=n            workgroup size of the composite passes (256, 512 or
 *                         1024) on every level, instead of the tuned choice
 *   AMGDD_LDS=1|0         the operator and restriction passes of every level
 *                         stage their tile's band of the gathered vector in
 *                         LDS / none does, instead of the tuned choice
 *   AMGDD_FUSED_R         restriction fused into the down pass with the
 *                         operator's row order and lanes (no reordered P, R)
 *   AMGDD_TIGHT_WINDOW=n  sort window of the reordered P and R (defaults 512
 *                         for P, 1024 for R); AMGDD_TIGHT_WINDOW_R=n for R only
 *   AMGDD_TILE_SLICES_MAX=n, AMGDD_WIDE_TILES_MIN=m  LDS tiles of a level's
 *                         operator hold the largest power of two of slices
 *                         from n (16 to 128, default 32) down that leaves the
 *                         level at least m tiles (default 0), else 16
 * and when a handle's schedule is tuned:
 *   AMGDD_TUNE_CACHE=path schedule cache file (JSON, one entry per line,
 *                         keyed by a hash of the layout, device and library
 *                         build); default $HOME/.cache/amgdd/schedules.json,
 *                         "off" = no file (the in-process cache remains)
 * Index width, LDS staging, the side-stream branch and the launch schedule
 * leave results bitwise unchanged; step width, row order, lanes per row and
 * the fused restriction change only the rounding of rows served by several
 * lanes.
 */
#ifndef AMGDD_H
#define AMGDD_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amgdd_ctx *amgdd_handle; /* opaque, owned by the library */

typedef enum {
  AMGDD_OK = 0,
  AMGDD_EINVAL = 1,       /* malformed input; nothing was modified */
  AMGDD_ENOMEM = 2,       /* host or device allocation failed */
  AMGDD_EDEVICE = 3,      /* HIP error, or a device call on a host-only handle */
  AMGDD_ENOCONV = 4,      /* maxit reached above rtol; x holds the last iterate */
  AMGDD_EBREAKDOWN = 5,   /* non-finite residual norm */
  AMGDD_EUNSUPPORTED = 6  /* valid input outside what the library supports */
} amgdd_status;

typedef enum { AMGDD_FP64 = 0, AMGDD_MIXED = 1 } amgdd_precision;

typedef struct {
  double theta;     /* strength threshold, default 0.25 */
  int max_coarse;   /* stop coarsening at <= this many points, default 16 */
  int max_levels;   /* default 25 */
  int padding;      /* eta_l on every level below the coarsest, default 1 */
  int n_fac;        /* AlgFAC cycles per AMG-DD iteration, default 2 */
  int precision;    /* amgdd_precision, default AMGDD_FP64 */
  int device;       /* HIP device ordinal; -1 = host-only handle (setup and
                       introspection only, every solve returns EDEVICE) */
  int use_graph;    /* 1 = replay each outer iteration as a HIP graph (default) */
  int tail_level;   /* AlgFAC schedule: levels >= tail_level run in one persistent
                       launch per cycle with one workgroup per composite grid,
                       levels above it level-synchronously over all grids.
                       -2 = chosen by the autotuner at the first solve (default;
                       the choice is cached per layout and device, see
                       AMGDD_TUNE_CACHE), -1 = level-synchronous everywhere,
                       >= 0 fixed */
  int tail_block;   /* workgroup size of the persistent launch: 256, 512 or 1024;
                       0 = chosen by the autotuner (default) */
  int hybrid_level; /* 0 = AMG-DD on the fine level (default).  L~ >= 1 = hybrid
                       AMG-DD (Algorithm 3): amgdd_solve runs hybrid V(1,1)
                       cycles whose coarse solver on level L~ is one AMG-DD
                       cycle (from zero, n_fac AlgFAC cycles) on A_L~ with the
                       subdomains inherited along the C-points (a coarse point
                       keeps the subdomain of its fine point, Section 5);
                       subdomains without points on L~ are dropped.  Composite
                       grids are built for the level-L~ problems only.  A
                       problem whose hierarchy ends at or above L~ runs plain
                       V(1,1) cycles (its level-L~ AMG-DD would be the direct
                       solve).  V-cycle levels run in FP64; `precision`
                       applies to the level-L~ AMG-DD cycle. */
  int relax_order;  /* 0 = l1-Jacobi in natural order, every point at once
                       (default); 1 = CF-ordered l1-Jacobi, the smoother of the
                       paper's experiments (Section 6): each relaxation is a
                       Jacobi half-sweep over the level's C-points and then one
                       over its F-points, the second seeing the first's update,
                       F-points first on the upsweep.  Applies to AlgFAC, the
                       V-cycle and the hybrid cycle alike. */
  int coarsen;      /* 0 = classical RS first pass (default); 1 = HMIS, the
                       coarsening of the paper's experiments (Section 6): one
                       RS first pass inside each subdomain, then PMIS (De
                       Sterck, Yang, Heys 2006) from its C-points that have no
                       strong connection to another subdomain; PMIS ties broken
                       by r_i = (SplitMix64(2^32 level + i) >> 11) / 2^53;
                       coarse-level subdomains inherited along the C-points */
  int interp;       /* 0 = direct interpolation (default); 1 = extended+i
                       interpolation (De Sterck, Falgout, Nolting, Yang 2008) */
  int interp_max;   /* extended+i rows keep their interp_max largest entries,
                       rescaled to the row's sum; 0 = no truncation; default 4 */
  int n_padding_levels;          /* length of padding_per_level; 0 (default) = none */
  const int *padding_per_level;  /* eta_l of Section 3 per level: level l < n_padding_levels
                                    is grown by padding_per_level[l] (>= 0), deeper levels by
                                    `padding`; the coarsest level is stored whole whatever
                                    its entry says.  Borrowed for the setup call only; NULL
                                    when n_padding_levels = 0.  Levels are counted from the
                                    fine level also on a hybrid handle. */
} amgdd_params;

typedef struct {
  int iters;            /* outer iterations (or V-cycles) performed */
  double relres;        /* max over problems of ||r_k|| / ||r_0|| */
  double rho_asym;      /* geometric-mean factor over the last <= 5 iterations */
  double solve_s;       /* host time of the solve from its first launch to the
                           synchronisation after its last iteration */
  double setup_s;       /* host setup time of the handle */
} amgdd_info;

typedef struct {
  int n_problems;
  int n_grids;              /* composite grids (subdomains) over all problems */
  int max_levels;           /* deepest hierarchy over all problems */
  long long fine_rows;      /* sum of N_0 */
  long long global_nnz;     /* sum over problems and levels of nnz(A_l) */
  long long composite_real_nnz; /* nnz of A_l rows at real points, all grids/levels */
  long long composite_rows;     /* sum over grids and levels of |Dbar_l| */
  long long composite_real_rows;/* sum over grids and levels of |D_l| */
  long long composite_stored_nnz;/* device nnz of composite A, P, R (incl. padding) */
  long long omissions;      /* interpolation entries dropped (Section 4.2) */
  double composite_overhead;/* composite_real_nnz / global_nnz (Section 6.1) */
  double setup_hierarchy_s; /* host time: strength, RS, interpolation, Galerkin */
  double setup_composite_s; /* host time: composite sets, local operators */
  double setup_pack_s;      /* host time: batched layouts */
  double setup_upload_s;    /* device allocation and upload */
  long long device_bytes;   /* device memory owned by the handle */
  int tail_level;           /* schedule in use (-1 level-synchronous; -2 not tuned yet) */
  int tail_block;
  double autotune_s;        /* time spent by the autotuner */
  long long composite_nnz;  /* nonzeros of composite A, P, R without padding */
  int hybrid_level;         /* transition level L~ of a hybrid handle, 0 otherwise.
                               n_grids, composite_* and omissions then describe
                               the level-L~ problems' grids (levels >= L~), and
                               composite_overhead = (nnz of A_l, l < L~, plus
                               composite_real_nnz) / global_nnz */
  int schedule_cached;      /* 1 = the schedule came from the schedule cache
                               (no tuning runs), 0 = tuned or fixed */
  int wide_levels;          /* bit l set: the level-synchronous passes of composite
                               level l run in 512-thread workgroups (chosen by the
                               autotuner), else 256 */
  int lds_levels;           /* bit l set: the level-synchronous passes with the
                               composite operator of level l run in 1024-thread
                               workgroups that stage the gathered vector's band in
                               LDS (chosen by the autotuner; same sums) */
  int restrict_lds_levels;  /* bit l set: the same for the restriction pass of
                               level l (the band of w_{l-1}) */
} amgdd_stats;

void amgdd_params_default(amgdd_params *prm);

/*
 * Build the AMG hierarchy and every subdomain's composite grid on the host,
 * then upload the batched device layout (unless prm->device == -1).
 *   n, rowptr[n+1], colind[nnz], val[nnz]: fine-grid matrix A_0, CSR, 0-based,
 *       int32 indices, columns sorted and unique in each row, a positive
 *       diagonal entry in every row.  The graph of A_0 must be symmetric.
 *   part[n]: subdomain of every fine point, values in [0, nparts), every
 *       subdomain non-empty (Omega_0^p of Section 3).
 *   prm: NULL for defaults.  hip_stream: hipStream_t (NULL = default stream).
 * Errors: EINVAL for malformed CSR / partition / parameters,
 *         EUNSUPPORTED for n <= max_coarse or a coarsest level > 1024 points.
 */
amgdd_status amgdd_setup_composite(int n, const int *rowptr, const int *colind, const double *val,
                                   const int *part, int nparts, const amgdd_params *prm,
                                   void *hip_stream, amgdd_handle *out);

/*
 * Batched form: nprob independent problems with their own matrices,
 * partitions and paddings, all composite grids of all problems in one
 * batched layout.  Fields of prm[0] other than the padding fields (theta,
 * max_coarse, max_levels, n_fac, precision, device, use_graph, ...) apply to
 * the whole batch; padding, n_padding_levels and padding_per_level are taken
 * per problem from prm[i].
 */
amgdd_status amgdd_setup_composite_batch(int nprob, const int *n, const int *const *rowptr,
                                         const int *const *colind, const double *const *val,
                                         const int *const *part, const int *nparts,
                                         const amgdd_params *prm, void *hip_stream,
                                         amgdd_handle *out);

/*
 * AMG-DD iterations (Algorithm 2 with n_fac AlgFAC cycles, Algorithm 4) on
 * A x = b; hybrid AMG-DD V-cycles (Algorithm 3) on a hybrid handle.  b_dev, x_dev: device FP64 vectors of length sum of N_0; x is the
 * initial guess on entry and the last iterate on return.  Stops when every
 * problem has ||b - A x|| <= rtol ||b - A x_0|| or after maxit iterations;
 * rtol <= 0 runs exactly maxit iterations and returns OK.  info may be NULL.
 */
amgdd_status amgdd_solve(amgdd_handle h, const double *b_dev, double *x_dev, double rtol, int maxit,
                         amgdd_info *info);

/*
 * For callers that cannot allocate device memory during a solve (serving
 * loops, harnesses that forbid hipMalloc): amgdd_solve's iterations with no
 * device allocation in the call -- no tuning runs (a handle whose schedule is
 * not tuned yet runs the level-synchronous schedule, which gives the same
 * iterates), no graph capture (kernels enqueued one by one), and the residual
 * partial sums and norms in a static device array of the library
 * (1 MiB per device: the handle must need at most 131072 doubles, one per 256
 * fine rows plus one per problem, i.e. about 33 million fine rows; larger
 * handles get EUNSUPPORTED with nothing run).  Every other array it uses was
 * allocated when the handle was set up.  Same arguments, stopping rule and
 * statuses as amgdd_solve.  Calls that overlap on one device share the static
 * array and race; it keeps the last call's contents, and every call writes
 * all of it that it reads.
 */
amgdd_status amgdd_solve_noalloc(amgdd_handle h, const double *b_dev, double *x_dev, double rtol, int maxit,
                                 amgdd_info *info);

/* AMG V(1,1) cycles (Algorithm 1) on the same hierarchy, same conventions. */
amgdd_status amgv_solve(amgdd_handle h, const double *b_dev, double *x_dev, double rtol, int maxit,
                        amgdd_info *info);

/*
 * Adjoint solve A^T lambda = g by AMG-DD iterations (hybrid cycles on a
 * hybrid handle) with the same hierarchy: the same C/F splittings, P_l,
 * R_l = P_l^T and composite grids.  Because A_{l+1} = R_l A_l P_l (Section 2),
 * A_{l+1}^T = R_l A_l^T P_l, so these form a Galerkin hierarchy for A^T whose
 * operators are the transposes A_l^T:
 *   - symmetric A_0 (checked bitwise at setup): A^T = A, the forward
 *     operators are used as they are;
 *   - otherwise the transposed composite operators (rows of A_l^T on every
 *     composite grid, l1-Jacobi diagonals sum_j |a_ji|, coarsest inverse of
 *     A_L^T) are built on the host and uploaded at the first adjoint call of
 *     the handle (host time and device memory comparable to the forward
 *     setup's composite part; reported in amgdd_stats.device_bytes), and
 *     kept until amgdd_destroy.
 * g_dev, lambda_dev: device FP64 of length sum N_0; lambda is in/out like
 * x_dev of amgdd_solve, with the same stopping rule and statuses.
 */
amgdd_status amgdd_solve_adjoint(amgdd_handle h, const double *g_dev, double *lambda_dev, double rtol,
                                 int maxit, amgdd_info *info);

/*
 * Face gradient of a loss through A(c) u = f with A = sum_f c_f E_f:
 *   interior face (i, j): dL/dc_f = -(lambda_i - lambda_j)(u_i - u_j)
 *   boundary face (i, -1): dL/dc_f = -lambda_i u_i
 * u_dev, lambda_dev: device FP64 of length sum N_0; face_i_dev, face_j_dev:
 * device int32 of length nfaces (j = -1 marks a boundary face; indices into
 * the concatenated vectors); dLdc_dev: device FP64 output of length nfaces.
 */
amgdd_status amgdd_face_gradient(amgdd_handle h, const double *u_dev, const double *lambda_dev,
                                 const int *face_i_dev, const int *face_j_dev, int nfaces,
                                 double *dLdc_dev);

/* ---- introspection (host copies into caller-allocated arrays) ---------- */

amgdd_status amgdd_get_stats(amgdd_handle h, amgdd_stats *st);

/* Level count and per-level sizes of problem prob (arrays of length >= nlevels;
 * pass NULL to query nlevels only). */
amgdd_status amgdd_get_levels(amgdd_handle h, int prob, int *nlevels, int *n_per_level,
                              long long *nnz_per_level);

/* C/F splitting of level `level` < nlevels-1: +1 C, -1 F, length N_level. */
amgdd_status amgdd_get_cf(amgdd_handle h, int prob, int level, signed char *cf);

/* Global operator of problem prob: which = 0 A_l, 1 P_l.  Call with NULL
 * arrays to get nrows/nnz, then again with rowptr[nrows+1], col[nnz], val[nnz]. */
amgdd_status amgdd_get_operator(amgdd_handle h, int prob, int level, int which, int *nrows, int *nnz,
                                int *rowptr, int *col, double *val);

/* Composite grid of subdomain p of problem prob on `level`: n_real = |D_l|,
 * n_bar = |Dbar_l|; gids (length n_bar, may be NULL) = global ids on that
 * level, real points first in increasing id, then ghost points in increasing
 * id; omissions = dropped interpolation entries for this grid and level.
 * Hybrid handle: levels >= hybrid_level only; EINVAL for a subdomain without
 * points on that level or a problem that has no level-L~ AMG-DD problem. */
amgdd_status amgdd_get_composite(amgdd_handle h, int prob, int p, int level, int *n_real, int *n_bar,
                                 int *gids, int *omissions);

/* Residual-norm history of problem prob from the last solve (length <= cap). */
amgdd_status amgdd_get_history(amgdd_handle h, int prob, double *hist, int cap, int *len);

/* Per-launch-site timing of the solve iteration (measurement only).
 * Runs `reps` iterations of kind 0 (AMG-DD, or hybrid on a hybrid handle;
 * levels of the level-L~ sites are counted from the fine level) or 1
 * (V-cycle) from the handle's
 * internal state, launching kernel by kernel (no graph) with a HIP event pair
 * around every launch on the handle's stream.  Sites are aggregated by
 * (kernel name, level): launches = launches per iteration, ms = device time
 * per iteration (median over the reps, so one stalled launch does not move
 * it), bytes = algorithmic bytes per iteration (stored nonzeros,
 * each vector entry touched once).  Fills up to cap entries of out, sets *n to
 * the number of sites. */
typedef struct {
  char name[24];
  int level;
  int launches;
  double ms;
  double bytes;
  int workgroups;   /* workgroups of the site's (last) launch */
  int block;        /* workgroup size */
} amgdd_kernel_time;

amgdd_status amgdd_profile(amgdd_handle h, int kind, int reps, amgdd_kernel_time *out, int cap, int *n);

/* Change the stream used by later calls. */
amgdd_status amgdd_set_stream(amgdd_handle h, void *hip_stream);

const char *amgdd_last_error(void);

/* Frees every device and host allocation of the handle; NULL is accepted. */
void amgdd_destroy(amgdd_handle h);

#ifdef __cplusplus
}
#endif

#endif /* AMGDD_H */
