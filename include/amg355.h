/*
 * amg355.h - C ABI of the MI355X (gfx950) smoothed-aggregation AMG library
 * (preconditioned CG and BiCGSTAB) with adjoint solves.
 *
 * What the calls compute (the paper delegates the numerical method to its
 * backend; the operations below are the ones its interface exposes):
 *   - a sparse solve A x = b returning x plus diagnostics (iterations, final
 *     residual, convergence status)                   -- Section 2.1/2.2
 *   - a setup cached per sparsity pattern; a cache hit with new values updates
 *     the coefficients in place and repeats the numeric setup -- Section 2.1
 *     ("C++/CUDA backend")
 *   - the adjoint solve A^T lambda = dL/dx            -- Eq. (1); a
 *     nonsymmetric A gets an explicit transpose A^T and its own hierarchy
 *     (Section 2.1)
 *   - BiCGSTAB with the AMG preconditioner, the paper's default solver for
 *     general (nonsymmetric) systems                  -- Section 2.1
 *   - the gradients dL/dA = -lambda x^T (restricted to the stored pattern)
 *     and dL/db = lambda                              -- Eq. (2)
 *   - single- and double-precision arithmetic         -- Section 2.2
 *
 * Conventions
 *   - Matrices are CSR: int32 row_ptr[n+1] (row_ptr[0] = 0,
 *     row_ptr[n] = nnz), int32 col[nnz] strictly ascending within a row and
 *     in [0, n), every row holding its diagonal; float64 values.
 *   - Every array argument is a DEVICE pointer owned by the caller.  The
 *     library copies what it keeps; it never frees caller memory.
 *   - All work is ordered on the given hipStream_t (pass the caller's current
 *     stream).  Calls that report sizes or statuses synchronise that stream.
 *   - A block of k right-hand sides is stored row-major: element (i, c) at
 *     [i*k + c].
 *   - Every entry point returns an amg_status; C++ exceptions never cross
 *     the ABI.  Non-convergence is a status (AMG_NOT_CONVERGED), not an
 *     error: x and the info block are still filled.
 *   - Handles are not thread-safe; calls that overlap on one handle race.
 */
#ifndef AMG355_H
#define AMG355_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amg_handle_s* amg_handle;

typedef enum {
  AMG_OK = 0,
  AMG_NOT_CONVERGED = 1,            /* maxiter reached; x holds the last iterate */
  AMG_ERR_INVALID_ARG = -1,         /* bad pointer/size/params or malformed CSR */
  AMG_ERR_ZERO_DIAG = -2,           /* a row has no stored or a zero diagonal */
  AMG_ERR_PATTERN_MISMATCH = -3,    /* value update with a different pattern */
  AMG_ERR_BREAKDOWN = -4,           /* p^T A p <= 0, r^T z <= 0, a zero BiCGSTAB scalar, NaN, or a
                                       non-SPD (symmetric) / singular (nonsymmetric) coarse matrix */
  AMG_ERR_OOM = -5,                 /* device allocation failed */
  AMG_ERR_HIP = -6,                 /* a HIP runtime call failed */
  AMG_ERR_COARSE_TOO_LARGE = -7,    /* coarsening stalled above the dense coarse-solve limit */
  AMG_ERR_SCRATCH_LIMIT = -8        /* the system exceeds the static workspace of amg_solve_noalloc */
} amg_status;

enum { AMG_PREC_FP64 = 0, AMG_PREC_FP32 = 1 };
enum { AMG_SMOOTHER_JACOBI = 0, AMG_SMOOTHER_L1 = 1 };
enum { AMG_CACHE_COLD = 0, AMG_CACHE_HIT = 1, AMG_CACHE_REFRESH = 2 };
enum { AMG_SOLVER_PCG = 0, AMG_SOLVER_BICGSTAB = 1 };

/* Largest coarsest level that receives a dense factorization (its explicit
 * inverse is applied once per cycle, m^2 values). */
#define AMG_MAX_DENSE_COARSE 2048
#define AMG_MAX_LEVELS 20

typedef struct {
  int vcycle_prec;     /* AMG_PREC_FP64 (default) or AMG_PREC_FP32 (FP32 V-cycle inside FP64 CG) */
  int transfer_bf16;   /* FP32 cycle only: P and R values stored as bfloat16 (default 1) */
  double theta;        /* strength threshold; 0 (default) = every off-diagonal entry is strong */
  int max_coarse;      /* stop coarsening at or below this many unknowns (default 256) */
  int max_levels;      /* at most this many levels (default 20, <= AMG_MAX_LEVELS) */
  int smoother;        /* AMG_SMOOTHER_JACOBI (default, weight omega/a_ii) or AMG_SMOOTHER_L1 */
  double omega;        /* Jacobi damping (default 2/3) */
  int nu_pre, nu_post; /* sweeps before/after the coarse correction (default 1, 1) */
  int maxiter;         /* Krylov iteration limit (default 1000) */
  int flexible;        /* -1 (default): flexible beta iff the cycle is not FP64 or nu_pre != nu_post (the
                          preconditioner is then not a fixed symmetric operator); 0 standard; 1 flexible */
  int symmetric;       /* 1 (default): A = A^T, the adjoint reuses A's hierarchy and the coarsest level
                          gets a Cholesky factorization.  0: A may be nonsymmetric (needs
                          solver = AMG_SOLVER_BICGSTAB): LU with partial pivoting on the coarsest level;
                          the adjoint forms A^T and builds its hierarchy on first use */
  int check_every;     /* PCG iterations queued between convergence checks (default 0 = automatic) */
  int use_graphs;      /* 1 (default): replay HIP-graph captured iterations (on a library stream
                          joined to the caller's stream by events); 0: launch every kernel */
  int autotune;        /* 1: time candidate kernel shapes per matrix at setup and keep the fastest
                          (cached across runs in $AMG_TUNE_CACHE if set); 0 (default): row-length rule */
  int precondition;    /* 1 (default): AMG V-cycle preconditioner; 0: no preconditioner (plain CG or
                          BiCGSTAB; the setup keeps level 0 only; one right-hand side and one system) */
  int solver;          /* AMG_SOLVER_PCG (default) or AMG_SOLVER_BICGSTAB (right-preconditioned
                          BiCGSTAB; one right-hand side and one system) */
  int fused_small;     /* 1 (default): a PCG solve of one right-hand side on a hierarchy small enough for
                          one compute unit (two levels, <= 1024 fine rows of <= 8 entries, dense coarsest
                          level <= 256 rows, FP64 V(1,1) cycle) runs as a single workgroup in one launch
                          (vectors in LDS, q = A p formed directly); 0: always the per-kernel path.  A
                          solve-time option (not part of the cache key) */
} amg_params;

typedef struct {
  int iters;           /* PCG: products A p performed; BiCGSTAB: full iterations (two products A y each;
                          a stop at the half step counts its iteration); sums over restarts */
  double rel_resid;    /* true ||b - A x||_2 / ||b||_2 in FP64 (max over columns for k > 1) */
  int status;          /* amg_status of the solve */
  int cache_event;     /* AMG_CACHE_COLD / HIT / REFRESH of the amg_setup that produced the handle */
  int restarts;        /* true-residual replacements performed */
  double setup_ms;     /* wall time of that setup or refresh */
  double solve_ms;     /* wall time of this solve (host clock, stream synchronised) */
} amg_info;

typedef struct {
  int num_levels;
  int64_t n[AMG_MAX_LEVELS];
  int64_t nnz[AMG_MAX_LEVELS];       /* nnz of A_l */
  int64_t nnz_p[AMG_MAX_LEVELS];     /* nnz of P_l = nnz of R_l (0 on the coarsest level) */
  int64_t nnz_g[AMG_MAX_LEVELS];     /* nnz of the strength graph of level l */
  double rho[AMG_MAX_LEVELS];        /* Gershgorin bound of rho(D^-1 A_l) */
  double omega_p[AMG_MAX_LEVELS];    /* prolongator damping (4/3)/rho */
  int mis_rounds[AMG_MAX_LEVELS];    /* rounds of the parallel independent-set selection */
  double operator_complexity;        /* sum nnz(A_l) / nnz(A_0) */
  int group_a[AMG_MAX_LEVELS];       /* lanes per row chosen for A_l, P_l, R_l kernels */
  int group_p[AMG_MAX_LEVELS];
  int group_r[AMG_MAX_LEVELS];
  int form_a[AMG_MAX_LEVELS];        /* sweep form over A_l: 0 lanes-per-row, 1 CSR-stream, 2 sliced */
  int64_t sliced_len[AMG_MAX_LEVELS]; /* stored entries of the sliced copy of A_l (0: none) */
  int single_workgroup;              /* 1: small enough for the one-workgroup PCG solve (fused_small) */
} amg_hier_stats;

/* Fields of a level that amg_export_field can copy out (for bit-exact checks). */
typedef enum {
  AMG_FIELD_AGG = 0,       /* int32[n_l]        aggregate of each node */
  AMG_FIELD_A_ROWPTR = 1,  /* int32[n_l+1] */
  AMG_FIELD_A_COL = 2,     /* int32[nnz_l] */
  AMG_FIELD_A_VAL = 3,     /* float64[nnz_l] */
  AMG_FIELD_A_VAL32 = 4,   /* float32[nnz_l]    (FP32 cycle) */
  AMG_FIELD_DINV = 5,      /* float64[n_l]      1 / a_ii */
  AMG_FIELD_P_ROWPTR = 6,  /* int32[n_l+1] */
  AMG_FIELD_P_COL = 7,     /* int32[nnz_p] */
  AMG_FIELD_P_VAL = 8,     /* float64[nnz_p] */
  AMG_FIELD_P_BF16 = 9,    /* uint16[nnz_p]     (FP32 cycle with bf16 transfers) */
  AMG_FIELD_R_ROWPTR = 10, /* int32[n_{l+1}+1] */
  AMG_FIELD_R_COL = 11,    /* int32[nnz_p] */
  AMG_FIELD_R_VAL = 12,    /* float64[nnz_p] */
  AMG_FIELD_R_BF16 = 13,   /* uint16[nnz_p] */
  AMG_FIELD_G_ROWPTR = 14, /* int32[n_l+1]      strength graph */
  AMG_FIELD_G_COL = 15,    /* int32[nnz_g] */
  AMG_FIELD_COARSE_FACTOR = 16, /* float64[m*m] factor of the coarsest A, row-major, m = padded size: Cholesky
                                   (lower) or, nonsymmetric, packed LU (unit-lower multipliers below the
                                   diagonal, U on and above) */
  AMG_FIELD_COARSE_INV = 17,    /* float64[m*m] inverse of the coarsest A, transposed (entry (j, i) holds
                                   (A^-1)_ij; equal to the inverse when A is symmetric) */
  AMG_FIELD_DINV32 = 18,   /* float32[n_l] smoother weights of the FP32 cycle */
  AMG_FIELD_COARSE_PIVOTS = 19, /* int32[m] nonsymmetric only: row exchanged with row k at LU step k */
  AMG_FIELD_SW = 20,            /* float64[n_l] smoother weights: omega/a_ii (damped Jacobi) or
                                   1/sum_j |a_ij| (L1-Jacobi) */
  AMG_FIELD_COARSE_INV32 = 21   /* float32[m*m] FP32 cycle: AMG_FIELD_COARSE_INV rounded to nearest even */
} amg_field;

/* Fills *p with the defaults listed above. */
void amg_params_default(amg_params* p);

/* Setup (Section 2.1, "C++/CUDA backend"): returns a handle to the hierarchy
 * of A = (row_ptr, col, val), n rows.  The library keeps an LRU cache keyed
 * by a 64-bit hash of (row_ptr, col, n, nnz, params) with a full pattern
 * compare on a hit.  Cold: full setup (strength graph, aggregation,
 * smoothed prolongator, R = P^T, Galerkin R A P per level, inverse
 * diagonals, coarse factorization).  Hit with identical values: the cached
 * hierarchy is returned.  Hit with new values: the values are refreshed in
 * place (aggregates and all patterns kept; with theta > 0 the strength graph
 * depends on the values, so the hierarchy is set up again from the pattern)
 * when no other caller's handle holds the hierarchy; when one does, that
 * hierarchy is left unchanged for it and a new one is built for the new
 * values and takes its place in the cache (copy on write).  A refresh that
 * fails part-way (AMG_ERR_ZERO_DIAG, AMG_ERR_BREAKDOWN, ...) drops the
 * hierarchy from the cache.  The handle holds one reference (release with
 * amg_destroy); the cache holds another.
 * n_systems = S >= 1 (at most 64): S systems share the pattern and d_val
 * holds their values interleaved, entry k of system s at [k*S + s]; the
 * aggregation is pattern-only (theta must be 0) and each system gets its own
 * numeric hierarchy.  *out is written only on success. */
amg_status amg_setup(const amg_params* params, int32_t n, int64_t nnz, const int32_t* d_row_ptr,
                     const int32_t* d_col, const double* d_val, int32_t n_systems, hipStream_t stream,
                     amg_handle* out);

/* Value refresh on the same pattern: recomputes every value of the hierarchy
 * from d_val (nnz entries) and keeps aggregates and patterns (theta > 0: sets
 * the hierarchy up again from the pattern).  In place when no other caller's
 * handle shares the hierarchy; otherwise this handle gets a hierarchy of its
 * own for the new values and the others keep theirs.  If the refresh fails
 * part-way, its status is returned, the hierarchy leaves the cache, and
 * amg_solve / amg_solve_adjoint / amg_apply_vcycle on it return that status
 * until a later amg_update_values succeeds. */
amg_status amg_update_values(amg_handle h, const double* d_val, hipStream_t stream);

/* Solve A X = B from X0 = 0 with the handle's solver.
 *
 * AMG_SOLVER_BICGSTAB (one system; nrhs > 1 columns of a row-major block
 * are solved one after another, with per-column outcomes in
 * amg_solve_columns and the maximum / worst in info): right-preconditioned BiCGSTAB
 * (y = M^-1 p, v = A y, s = r - alpha v, z = M^-1 s, t = A z), shadow residual
 * r^ = b, scalars formed on the device.  Stops when the recursive ||s||_2 or
 * ||r||_2 <= tol ||b||_2, verifies the true residual and restarts from it
 * (at most 5 times) like PCG.  A zero or NaN rho, <r^, v>, <t, t> or omega is
 * AMG_ERR_BREAKDOWN.
 *
 * AMG_SOLVER_PCG: PCG for nrhs >= 1 columns (row-major blocks,
 * nrhs <= 64), preconditioned by one V-cycle per iteration.  With n_systems
 * S > 1, nrhs must equal S and column s is solved with system s.  Columns are
 * independent CG iterations run in one batched launch per step (not block
 * CG); converged columns are frozen.  Batched solves need at least two
 * levels and V(1,1); info reports the maximum iteration count and residual
 * over the columns and the worst status (see amg_solve_columns).  Stops when
 * ||r||_2 <= tol ||b||_2 for the recursive residual, then verifies the true
 * residual in FP64 and restarts from it (at most 5 times) if it misses.
 * tol = 0 runs exactly params.maxiter iterations.  info may be null. */
amg_status amg_solve(amg_handle h, const double* d_b, double* d_x, double tol, int32_t nrhs, amg_info* info,
                     hipStream_t stream);

/* Adjoint solve A^T lambda = g (Eq. (1)) with the same solver, precision and
 * tolerance rule as amg_solve.  symmetric = 1: A's own hierarchy is the
 * hierarchy of A^T and no transpose is formed.  symmetric = 0 (BiCGSTAB, its
 * column rule for nrhs > 1): the
 * first call forms A^T on the device (stable radix sort of the entries by column) and
 * sets up its hierarchy with the same parameters; both are kept with the
 * handle and refreshed from A's values after a value update. */
amg_status amg_solve_adjoint(amg_handle h, const double* d_g, double* d_lambda, double tol, int32_t nrhs,
                             amg_info* info, hipStream_t stream);

/* Per-column outcome of the handle's last batched solve (ncols = its width):
 * iterations, true relative residual and status of every column. */
amg_status amg_solve_columns(amg_handle h, int32_t ncols, int* iters, double* rel_resid, int* status);

/* Pattern gradient (Eq. (2)): grad_val[k] = -(lambda[row k] * x[col k]) for
 * every stored entry k of the level-0 matrix; dL/db is lambda itself. */
amg_status amg_pattern_grad(amg_handle h, const double* d_lambda, const double* d_x, double* d_grad_val,
                            hipStream_t stream);

/* Batched pattern gradient for ncols columns ([n][ncols] lambda and x):
 * with S systems, grad_val is [nnz][S] (per system); with one matrix and
 * ncols right-hand sides, grad_val[k] sums -(lambda_c[row k] x_c[col k]) over
 * the columns in ascending order (the gradient with respect to the shared
 * values of a loss over all columns). */
amg_status amg_pattern_grad_batched(amg_handle h, const double* d_lambda, const double* d_x, int32_t ncols,
                                    double* d_grad_val, hipStream_t stream);

/* One V-cycle z = M^-1 r on the fine level (FP64 in and out, the handle's
 * cycle precision inside): the preconditioner as an operator. */
amg_status amg_apply_vcycle(amg_handle h, const double* d_r, double* d_z, hipStream_t stream);

/* Allocation-free PCG solve, for callers that cannot allocate device memory
 * (code recorded under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  It computes what amg_solve(h, d_b, d_x, tol, 1, info,
 * stream) computes with use_graphs = 0 -- the same kernels in the same order,
 * so the same x bit for bit -- but its Krylov workspace (residual r,
 * preconditioned residual z, the two direction buffers, q = A p, the
 * per-workgroup partial sums and the device control block) lives in one
 * static device array of AMG_NOALLOC_SCRATCH_BYTES per GPU instead of the
 * handle's buffers.  That array is part of the library's code object: each
 * GPU the library runs on holds it from the library's load until the
 * process ends.  The call makes no hipMalloc, hipFree, graph or other
 * allocating call; it synchronises the stream between iteration chunks like
 * amg_solve.  Each call clears the part of the array that must start at
 * zero; contents otherwise persist from the previous call.
 * Limits: a PCG handle (solver = AMG_SOLVER_PCG) of one system, one
 * right-hand side, n <= AMG_NOALLOC_MAX_N rows and at most
 * AMG_NOALLOC_MAX_PARTIALS partial-sum slots (level-0 sweep grids of a few
 * hundred thousand workgroups); a larger system returns
 * AMG_ERR_SCRATCH_LIMIT before anything is launched, another solver or width
 * AMG_ERR_INVALID_ARG.  Every call on a GPU uses that GPU's one array: calls
 * that overlap on one GPU (any handles, any streams, any threads) race and
 * must be serialised by the caller. */
#define AMG_NOALLOC_MAX_N 2097152
#define AMG_NOALLOC_MAX_PARTIALS 1048576
#define AMG_NOALLOC_SCRATCH_BYTES (256 + 8 * (size_t)AMG_NOALLOC_MAX_PARTIALS + 5 * 8 * (size_t)AMG_NOALLOC_MAX_N)
amg_status amg_solve_noalloc(amg_handle h, const double* d_b, double* d_x, double tol, amg_info* info,
                             hipStream_t stream);

/* ---- matrix-free operators (Section 2.1, "Matrix-free operator support") ----
 * An operator given as a callable x -> A x with a known CSR pattern is
 * materialized by graph-colored probing (Curtis-Powell-Reid): the columns are
 * colored so that no two columns of a color share a row, the operator is
 * applied once to each color's 0/1 probe vector, and every stored entry is
 * read off the products: a_ij = (A v_color(j))_i.  The caller applies the
 * operator (it is the caller's code); the library colors, builds the probes
 * and assembles.  Probe and product blocks are stored [ncolors][n] (one
 * contiguous vector per color).  The pattern follows the CSR conventions
 * above (sorted columns, every diagonal stored) and is validated.
 *
 * Coloring: greedy in decreasing node-key order (the keys of the
 * aggregation), each column taking the smallest color not used by an
 * already colored column that shares a row with it; deterministic.
 * d_color: int32[n] device output; *ncolors: host output (the stream is
 * synchronised). */
amg_status amg_color_columns(int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col,
                             int32_t* d_color, int32_t* ncolors, hipStream_t stream);

/* d_V (float64[ncolors*n], device): V[c*n + j] = 1 if color[j] == c, else 0.
 * A color outside [0, ncolors) is AMG_ERR_INVALID_ARG (nothing written). */
amg_status amg_probe_vectors(int32_t n, const int32_t* d_color, int32_t ncolors, double* d_V, hipStream_t stream);

/* d_val[k] = d_Y[color[col k]*n + row k] for every stored entry k, where d_Y
 * (float64[ncolors*n]) holds the products A V_c.  Exact (no arithmetic): the
 * result equals A's values when the pattern covers A's nonzeros. */
amg_status amg_probe_assemble(int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col,
                              const int32_t* d_color, int32_t ncolors, const double* d_Y, double* d_val,
                              hipStream_t stream);

/* Adjoint of amg_probe_assemble (for gradients through the operator):
 * d_dY = 0, then d_dY[color[col k]*n + row k] = d_dval[k]. */
amg_status amg_probe_scatter(int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col,
                             const int32_t* d_color, int32_t ncolors, const double* d_dval, double* d_dY,
                             hipStream_t stream);

/* Hierarchy statistics (Section 2.2 diagnostics). */
amg_status amg_hierarchy_stats(amg_handle h, amg_hier_stats* out);

/* Size in elements and bytes per element of a level field. */
amg_status amg_field_info(amg_handle h, int level, int field, int64_t* count, int* elem_bytes);

/* Device-to-device copy of a level field into d_dst (dst_bytes capacity). */
amg_status amg_export_field(amg_handle h, int level, int field, void* d_dst, size_t dst_bytes, hipStream_t stream);

/* ---- measurement (diagnostics; no effect on results) ----
 * Kernel ids for amg_instrument / amg_kernel_bytes. */
enum {
  AMG_KERNEL_SPMV_DOT = 0,   /* p = z + beta p, q = A z + beta q (= A p), <p,q> (level 0, one fused sweep) */
  AMG_KERNEL_PRE = 1,        /* residual of the pre-smoothed iterate x = sw o b */
  AMG_KERNEL_POST = 2,       /* post-smoothing sweep (level 0: writes z, reduces <r,z>) */
  AMG_KERNEL_RESTRICT = 3,   /* b_{l+1} = R_l r_l */
  AMG_KERNEL_PROLONG = 4,    /* x_l += P_l x_{l+1} */
  AMG_KERNEL_CG_UPDATE = 5,  /* x += alpha p, r -= alpha q, <r,r>, x0 = sw o r */
  AMG_KERNEL_XPAY = 6,       /* (fused into AMG_KERNEL_SPMV_DOT; never launched) */
  AMG_KERNEL_COARSE = 7      /* dense coarsest solve */
};

/* Time every launch of one kernel at one level (level -1: all levels)
 * inside subsequent solves with HIP event pairs on the solve stream
 * (kernel -1 switches it off).  Resets the record. */
amg_status amg_instrument(amg_handle h, int kernel, int level);

/* Synchronises on the recorded events; returns the number of timed launches
 * that did work and their total, minimum and maximum durations in ms.
 * Launches that started after the solve had converged (they return at once)
 * are left out. */
amg_status amg_instrument_read(amg_handle h, int* launches, double* total_ms, double* min_ms, double* max_ms);

/* Algorithmic bytes of one launch of `kernel` at `level` (every matrix
 * array streamed once, every vector operand read once, every output written
 * once); kernel -1: one whole PCG iteration.  flexible: 1 if the solve uses
 * the flexible beta (adds the read of q to the level-0 post-smoother). */
amg_status amg_kernel_bytes(amg_handle h, int kernel, int level, int flexible, double* bytes);

/* Algorithmic bytes of one launch of a batched sweep with `width` columns
 * (amg_solve with nrhs = width; with n_systems S > 1, width must be S): the
 * batched kernels stream every operator as CSR (int32 columns and row
 * pointers, once per launch); values, smoother weights and coarse inverses
 * are read once per launch for right-hand sides of one matrix and once per
 * column for S systems sharing a pattern; every vector operand is width
 * columns wide.  kernel -1: one whole batched PCG iteration with every column
 * active.  amg_instrument times the batched solve's launches the same way
 * (the done test is then "every column finished"). */
amg_status amg_kernel_bytes_batched(amg_handle h, int kernel, int level, int flexible, int32_t width,
                                    double* bytes);

/* Releases the caller's reference; the hierarchy is freed when neither a
 * caller nor the cache holds it. */
amg_status amg_destroy(amg_handle h);

/* Empties the setup cache (Section 3.4 "finalize"). Handles still held by
 * callers stay valid until destroyed. */
amg_status amg_finalize(void);

/* Number of hierarchies currently in the cache; capacity setter (default 8). */
int amg_cache_size(void);
amg_status amg_set_cache_capacity(int capacity);

/* The rounding of the bf16-stored transfer operators of the FP32 cycle
 * (Section 2.2 single precision; storage only): d_out[i] = the bfloat16
 * nearest to d_in[i], ties to even; every NaN becomes the quiet NaN 0x7fc0.
 * d_in: float32[n], d_out: uint16[n] (bfloat16 bit patterns), both device
 * pointers owned by the caller; n = 0 writes nothing.  Stream-ordered, no
 * synchronisation. */
amg_status amg_convert_bf16(const float* d_in, uint16_t* d_out, int64_t n, hipStream_t stream);

/* Human-readable name of a status. */
const char* amg_status_string(amg_status s);

#ifdef __cplusplus
}
#endif

#endif /* AMG355_H */
