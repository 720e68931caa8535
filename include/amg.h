/*
 * amg.h - C interface of the MI355X (gfx950) aggregation AMG-preconditioned CG.
 *
 * The method is the non-smoothed aggregation algebraic multigrid of Blatt,
 * Ippisch and Bastian ("A Massively Parallel Algebraic Multigrid
 * Preconditioner based on Aggregation for Elliptic Problems with
 * Heterogeneous Coefficients"): strength of connection and greedy
 * aggregation (Sec. 2.1, Alg. 1-3) run decoupled per tile of rows (Sec. 3.3,
 * Alg. 4), piecewise-constant prolongation and the Galerkin coarse operator
 * (Sec. 2.1, eq. (prolongation)), and a V-cycle (Sec. 2) used as the
 * preconditioner of a conjugate-gradient solve of A x = b (Sec. 2, eq. (ls)).
 *
 * Conventions for every call:
 *  - Array pointers are HIP DEVICE pointers unless the comment says "host".
 *  - `stream` is a hipStream_t passed as void*; NULL selects the null stream.
 *    All device work of a call is enqueued on that stream.
 *  - Every call returns a status; on failure nothing leaks, output handles
 *    are set to NULL, and a message is available from amg_last_error()
 *    (per thread).  Errors of asynchronous kernels surface at the next
 *    synchronising call as AMG_ERR_HIP.
 *  - CSR matrices use int32 row pointers and columns (ascending within each
 *    row, diagonal stored, no duplicates) and float64 values, and must be
 *    structurally symmetric.
 */
#ifndef AMG_MI355X_AMG_H
#define AMG_MI355X_AMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define AMG_API __attribute__((visibility("default")))
#else
#define AMG_API
#endif

typedef enum amg_status {
  AMG_OK = 0,
  AMG_ERR_INVALID_ARG = 1,        /* malformed CSR or argument                        */
  AMG_ERR_BAD_DIAGONAL = 2,       /* missing diagonal or a_ii <= 0                   */
  AMG_ERR_NOT_SYMMETRIC = 3,      /* a_ij != a_ji (when check_symmetry is set)       */
  AMG_ERR_NOT_SPD = 4,            /* coarsest Cholesky pivot <= 0                     */
  AMG_ERR_COARSENING_STALLED = 5, /* coarsest level larger than 4096 rows             */
  AMG_ERR_OUT_OF_MEMORY = 6,
  AMG_ERR_BREAKDOWN = 7,          /* CG: p^T A p <= 0 or r^T z <= 0                   */
  AMG_ERR_NOT_CONVERGED = 8,      /* maxit reached; x holds the last iterate          */
  AMG_ERR_HIP = 9,                /* a HIP runtime call failed                        */
  AMG_ERR_UNSUPPORTED = 10        /* parameter outside what the kernels support       */
} amg_status;

/* Sparse SPD matrix A (Sec. 2, eq. (ls)), device CSR.  The library copies it
 * during amg_setup; the caller may free it afterwards. */
typedef struct amg_csr {
  int32_t n;              /* rows = columns, > 0                              */
  int32_t nnz;            /* stored entries = rowptr[n]                       */
  const int32_t *rowptr;  /* device, n+1                                      */
  const int32_t *colind;  /* device, nnz, ascending per row                   */
  const double *vals;     /* device, nnz                                      */
} amg_csr;

/* Smoothers: multicolour symmetric Gauss-Seidel over the whole level;
 * l1-Jacobi; the paper's hybrid symmetric Gauss-Seidel (Sec. 3.2: block-
 * Jacobi over smoothing tiles of smooth_tile_rows rows, one sequential forward +
 * backward Gauss-Seidel sweep inside each tile, levels kept in natural order); the
 * same hybrid form with each tile's rows swept colour by colour (colour, then
 * row; the colours a first-fit colouring of each tile on its own, rows
 * ascending, couplings inside the tile only), which runs a level's whole
 * symmetric step in one launch: one workgroup per tile, one step per colour
 * and direction (for coarse levels, where the multicolour smoother's two
 * launches per colour are latency bound). */
enum {
  AMG_SMOOTHER_MCSGS = 0,
  AMG_SMOOTHER_L1_JACOBI = 1,
  AMG_SMOOTHER_HYBRID_SGS = 2,
  AMG_SMOOTHER_TILE_MCSGS = 3
};

/* Parameters.  Defaults from amg_default_params() in brackets. */
typedef struct amg_params {
  double strength_threshold; /* delta of eq. (symmetric_strong2)               [0.08] */
  double isolated_threshold; /* beta: eta_max(i) < beta marks i isolated       [1e-5] */
  int32_t agg_min;           /* s_min of Alg. 2                                [8]    */
  int32_t agg_max;           /* s_max of Alg. 3 (at most 32)                   [12]   */
  int32_t agg_diameter;      /* d_max of Alg. 2 (at least 1)                   [3]    */
  double omega;              /* over-correction of the coarse correction       [1.6]  */
  int32_t coarse_max;        /* stop coarsening at <= this many rows           [500]  */
  int32_t max_levels;        /*                                                [25]   */
  int32_t tile_rows;         /* rows per decoupled aggregation tile (64..1024) [128]  */
  int32_t smoother;          /* AMG_SMOOTHER_*                                 [MCSGS]*/
  int32_t pre_sweeps;        /* symmetric GS steps (fwd+bwd) or Jacobi sweeps  [1]    */
  int32_t post_sweeps;       /*                                                [1]    */
  int32_t vcycle_fp32;       /* 1: V-cycle in FP32 on levels 0..L-1            [0]    */
  int32_t flexible;          /* 1: flexible CG (Polak-Ribiere beta); -1: = vcycle_fp32 [-1] */
  uint32_t colour_seed;      /* seed of the colouring priorities               [0]    */
  int32_t check_symmetry;    /* 1: reject A with a_ij != a_ji                  [1]    */
  int32_t keep_setup_data;   /* 1: keep strong/isolated flags for amg_copy_level [0]  */
  int32_t use_graphs;        /* 1: pcg_solve replays each iteration as a HIP   [1]
                                graph (systems below 1.5M rows x right-hand sides;
                                larger ones launch directly, which is as fast) */
  int32_t tail_rows;         /* levels with at most this many rows (and all    [0]
                                coarser ones) are cycled by one workgroup per solve */
  int32_t colour_tile_rows;  /* rows per tile of the colouring order of the    [128]
                                multicolour levels (64..1024)                      */
  int32_t block_size;        /* unknowns per node, 1..4 (point-based AMG for    [1]
                                systems, Sec. 4.2): A is given in scalar form with
                                node i's unknowns in rows i*bs .. i*bs+bs-1 and
                                every stored bs x bs block stored in full (the
                                diagonal block included).  Strength (with the
                                row-sum norms of the blocks as the weights of
                                Sec. 2.1), aggregation and colouring run on the
                                node graph; P = P_nodes (x) I; the smoother is
                                the multicolour block symmetric Gauss-Seidel
                                with inverted diagonal blocks (smoother must be
                                MCSGS, tail_rows 0).  With keep_setup_data the
                                strong / isolated flags of amg_copy_level are
                                those of the node graph. */
  int32_t spmv_format;       /* level-0 outer product of CG: 0 SELL-64 slices   [0]
                                (one lane per row); 1 CSR with a group of lanes per
                                row (keeps the level's CSR arrays, 12 B per entry) */
  int32_t coarse_smoother;   /* AMG_SMOOTHER_* of levels coarse_from and below;  [-1]
                                -1: `smoother` on every level */
  int32_t coarse_from;       /* first level of coarse_smoother and of         [1]
                                coarse_smooth_tile_rows (>= 1 when either is set) */
  int32_t smooth_tile_rows;  /* rows per block of the tile smoothers          [0]
                                (HYBRID_SGS, TILE_MCSGS: the blocks of the block-
                                Jacobi of Sec. 3.2) on levels above coarse_from;
                                64..1024, 0: tile_rows.  Independent of the
                                aggregation tiles: a block may span several of
                                them or split one. */
  int32_t coarse_smooth_tile_rows; /* the same from level coarse_from on;     [0]
                                0: as on the finer levels */
} amg_params;

typedef struct amg_solve_info {
  int32_t iterations;
  int32_t converged;          /* 1 if ||r||/||r0|| <= rtol                           */
  int32_t levels;
  double rel_residual;        /* recursive ||r_k|| / ||r_0||                         */
  double true_rel_residual;   /* ||b - A x|| / ||b|| in FP64                         */
  double setup_ms;            /* of the hierarchy used                               */
  double solve_ms;
} amg_solve_info;

typedef struct amg_hierarchy amg_hierarchy; /* opaque, library-owned */

/* Fills *p with the defaults listed above. */
AMG_API amg_status amg_default_params(amg_params *p);

/* Builds the AMG hierarchy of A (Sec. 2.1 and Sec. 3.3): per level, strength
 * of connection (eqs. (symmetric_strong1), (symmetric_strong2)), greedy
 * aggregation per tile of `tile_rows` rows (Alg. 1-4), numbering of the coarse
 * rows, Galerkin product P^T A P (stored unscaled; omega is applied at
 * prolongation), multicolouring for the smoother, optional FP32 copies; the
 * coarsest level (<= coarse_max rows) is factorised by a dense FP64 Cholesky.
 * Validates A first (INVALID_ARG, BAD_DIAGONAL, NOT_SYMMETRIC).  Blocks until
 * the hierarchy is complete.  *out receives the handle (NULL on failure).
 * The colourings and the coarsest factorisation run on a second host thread
 * with a stream of its own (started and joined inside the call), beside the
 * coarsening on `stream`. */
AMG_API amg_status amg_setup(const amg_csr *A, const amg_params *p, void *stream, amg_hierarchy **out);

/* One V-cycle z = M r (Sec. 2): pre-smoothing, residual restriction with P^T,
 * recursion, coarsest solve, prolongation with omega, post-smoothing.
 * r and z are device vectors of length n (level 0) and must not alias.
 * Asynchronous: returns after enqueueing. */
AMG_API amg_status amg_precond_apply(amg_hierarchy *h, const double *r, double *z, void *stream);

/* amg_precond_apply for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same launches and the same result bit for bit, with the
 * V-cycle's vectors (level-0 r and z in solve order; per level the iterate,
 * right-hand side and residual, in the cycle's precision) taken from a fixed
 * file-scope array of 64 MiB per device instead of the allocator.  No device
 * memory is allocated or freed by the call.  A hierarchy whose vectors need
 * more than 64 MiB (about 27 B per level-0 row in FP64, 30 B with the FP32
 * cycle: up to about 2.2 M rows) or that uses the one-workgroup tail
 * (tail_rows > 0) is rejected with AMG_ERR_UNSUPPORTED before any work is
 * enqueued.  Every call on one device shares that device's array, which
 * keeps the last call's contents (every value a cycle reads is written by it
 * first): calls that overlap on one device, on any streams, race and must be
 * ordered by the caller.  Asynchronous on `stream`; the caller synchronises
 * that stream before amg_free of the hierarchy. */
AMG_API amg_status amg_precond_apply_noalloc(amg_hierarchy *h, const double *r, double *z, void *stream);

/* Preconditioned CG (flexible CG if the hierarchy was built with flexible=1)
 * for A x = b with x holding x0 on entry and the solution on return.  Stops
 * when ||r_k||_2 <= rtol ||r_0||_2 (recursive residual) or after maxit
 * iterations (then AMG_ERR_NOT_CONVERGED with x = last iterate and *info
 * filled).  Blocks until done.  The iterations run on a stream owned by the
 * hierarchy's solve context (created on first use), ordered after the
 * caller's earlier work on `stream`; with use_graphs (and below 1.5M rows)
 * each iteration from the second on is one replay of a captured HIP graph.
 * Calls on one hierarchy
 * (pcg_solve, bicgstab_solve, amg_precond_apply) must not overlap.
 *   info      host, nullable
 *   res_hist  host, nullable, maxit+1 doubles: ||r_k||/||r_0||
 *   iter_hist device, nullable, n*(maxit+1) doubles: x_k for k = 0.. */
AMG_API amg_status pcg_solve(amg_hierarchy *h, const double *b, double *x, double rtol, int32_t maxit,
                     amg_solve_info *info, double *res_hist, double *iter_hist, void *stream);

/* BiCGSTAB (van der Vorst 1992), the outer solver of the paper's experiments
 * (Sec. 5, which applies the preconditioner twice per iteration), right-
 * preconditioned by one V-cycle of h for each of the two directions p and s.
 * x holds x0 on entry and the solution on return.  Vectors, errors, streams
 * and blocking as in pcg_solve (one iteration per host round trip; no graph).
 * BiCGSTAB assumes a fixed preconditioner: with vcycle_fp32 the cycle's
 * rounding makes it vary slightly, and the iteration can stall just above a
 * tight rtol (observed near 2.5e-8 for 1e-8 on one 256^3 system); the FP64
 * cycle, or flexible CG for the FP32 cycle, avoids that.
 * Each call takes 5 n + 16 K doubles of device memory through the allocator
 * (r, r~, p, v, t, partial sums) beyond the solve context's vectors and
 * returns them before it returns.
 * The stop test ||.||_2^2 <= (rtol ||r_0||_2)^2 is made on s (half step: x =
 * x_{k-1} + alpha M p, *half_step = 1) and on r_k; info->iterations is the
 * iteration k it stopped in.  AMG_ERR_BREAKDOWN when r~.v, t.t, omega or r~.r
 * is zero or not finite before convergence (x = the iterate at that point).
 *   half_step host, nullable
 *   res_hist  host, nullable, maxit+1 doubles: ||r_k||/||r_0|| (||s_k||/||r_0||
 *             for a half-step exit)
 *   iter_hist device, nullable, n*(maxit+1) doubles: x_k for k = 0.. */
AMG_API amg_status bicgstab_solve(amg_hierarchy *h, const double *b, double *x, double rtol, int32_t maxit,
                                  amg_solve_info *info, int32_t *half_step, double *res_hist, double *iter_hist,
                                  void *stream);

/* Releases everything the hierarchy owns.  NULL-safe.  Waits until the last
 * amg_precond_apply on the hierarchy has finished on its stream before any
 * memory is handed back.  The hierarchy must not be part of a running batch
 * entry (amg_batch_submit). */
AMG_API void amg_free(amg_hierarchy *h);

/* ---- many systems -------------------------------------------------------- */
/* Builds the hierarchies of nsys independent systems A[0..nsys) with one
 * parameter set (each system as in amg_setup).  The setups run concurrently
 * (host threads, one stream each) and overlap on the device.  Blocks until
 * all are complete.  out: host array of nsys handles; on failure every handle
 * is NULL and the status is that of the first failing system. */
AMG_API amg_status amg_setup_batched(const amg_csr *A, int32_t nsys, const amg_params *p, void *stream,
                                     amg_hierarchy **out);

/* Solves nsys systems with nrhs right-hand sides each (nrhs = 1, 2, 4 or 8)
 * by (flexible) preconditioned CG as in pcg_solve, all of them advanced
 * together: every step is one launch per kernel for all systems (the V-cycle
 * level by level, the CG vector updates), so the matrix of a system is read
 * once for its nrhs right-hand sides.  b[s] and x[s] are device arrays of
 * nrhs * n_s doubles, right-hand side k at offset k * n_s; x[s] holds x0 on
 * entry.  Each right-hand side stops at its own convergence (its iterate is
 * then frozen); its result equals that of pcg_solve alone bit for bit when
 * nrhs = 1 (and has the same arithmetic for any nrhs).  The hierarchies must
 * share vcycle_fp32, smoother, sweeps and the CG variant.  info: host, nullable,
 * nsys * nrhs records (system-major).  Returns AMG_OK if every right-hand side
 * converged, else AMG_ERR_BREAKDOWN or AMG_ERR_NOT_CONVERGED.  Blocks. */
AMG_API amg_status pcg_solve_batched(amg_hierarchy *const *h, int32_t nsys, int32_t nrhs, const double *const *b,
                                     double *const *x, double rtol, int32_t maxit, amg_solve_info *info,
                                     void *stream);

/* ---- continuous batching ------------------------------------------------- */
/* A batch holds up to max_entries running solves (entries) of nrhs
 * right-hand sides each.  amg_batch_submit adds a solve of hierarchy h
 * (vectors as in pcg_solve_batched, ordered after earlier work on `stream`);
 * it joins the running ones at the next step.  amg_batch_step performs
 * `iterations` CG iterations of every running entry; entries that finish are
 * completed (true residual computed, x written) inside the step and reported
 * by amg_batch_poll (tags, status, info: host, nrhs records per entry, up to
 * cap entries, *count returned).  An entry's arithmetic does not depend on
 * the other entries.  Submitting to a full batch returns AMG_ERR_INVALID_ARG.
 * One host thread per batch. */
typedef struct amg_batch amg_batch;
AMG_API amg_status amg_batch_create(int32_t nrhs, int32_t max_entries, int32_t use_graphs, amg_batch **out);
AMG_API amg_status amg_batch_submit(amg_batch *b, amg_hierarchy *h, const double *rhs, double *x, double rtol,
                                    int32_t maxit, int64_t tag, void *stream);
AMG_API amg_status amg_batch_step(amg_batch *b, int32_t iterations);
AMG_API amg_status amg_batch_poll(amg_batch *b, int64_t *tags, amg_status *status, amg_solve_info *info,
                                  int32_t cap, int32_t *count);
/* Entries submitted and not yet polled-out as finished. */
AMG_API amg_status amg_batch_active(const amg_batch *b, int32_t *active);
/* Device bytes of the running entries' vectors. */
AMG_API amg_status amg_batch_bytes(const amg_batch *b, size_t *bytes);
AMG_API void amg_batch_free(amg_batch *b);

/* ---- support ---------------------------------------------------------- */
AMG_API const char *amg_status_string(amg_status s);
AMG_API const char *amg_last_error(void);

/* Device allocator used for all library memory.  Default: a cache of
 * hipMalloc blocks (freed blocks are reused best fit, by the stream that
 * freed them, or by any stream once the library has synchronised that stream
 * after the free; idle blocks return to the device only when a hipMalloc
 * fails).
 * alloc returns NULL on
 * failure.  Passing NULL for both restores the default.  Change it only while
 * no hierarchy, batch or solve allocated by the other allocator exists and
 * no call is running. */
typedef void *(*amg_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*amg_free_fn)(void *ptr, void *stream, void *ctx);
AMG_API amg_status amg_set_allocator(amg_alloc_fn alloc, amg_free_fn free_fn, void *ctx);

/* Returns the default allocator's cached blocks on the current device (memory
 * of freed hierarchies, solve contexts and batches, kept for reuse) to the
 * device, after synchronising the device.  Memory in use is not affected.
 * Call it while no other call of the library is running, for instance before
 * handing the memory to another allocator. */
AMG_API amg_status amg_release_cached_memory(void);

/* Device bytes held by the hierarchy. */
AMG_API amg_status amg_hierarchy_bytes(const amg_hierarchy *h, size_t *bytes);

/* Device memory estimate (upper estimate for 7-point-like operators with
 * aggregates of 8-12 rows; grows with coarse-level fill for denser
 * matrices) for a hierarchy of an n x n matrix with nnz entries under
 * parameters p: peak during amg_setup, held by the hierarchy afterwards, and
 * held by one solve with nrhs right-hand sides (each output nullable).  No
 * device work; used for admission by memory footprint. */
AMG_API amg_status amg_estimate_bytes(int32_t n, int32_t nnz, const amg_params *p, int32_t nrhs,
                                      size_t *setup_peak, size_t *hierarchy, size_t *context);

/* Number of levels (level 0 is the input matrix). */
AMG_API amg_status amg_num_levels(const amg_hierarchy *h, int32_t *levels);

/* Shape of level l: rows, stored entries, colours, rows of level l+1 (0 on
 * the coarsest level). */
AMG_API amg_status amg_level_info(const amg_hierarchy *h, int32_t l, int32_t *n, int32_t *nnz, int32_t *ncolours,
                          int32_t *n_next);

/* Copies level l to HOST arrays (each nullable): aggregate id per row (n; not
 * on the coarsest level), colour per row (n), CSR (n+1, nnz, nnz), and, when
 * built with keep_setup_data, the strong flag per stored entry (nnz) and the
 * isolated flag per row (n).  Synchronises the null stream. */
AMG_API amg_status amg_copy_level(const amg_hierarchy *h, int32_t l, int32_t *agg, int32_t *colour, int32_t *rowptr,
                          int32_t *colind, double *vals, uint8_t *strong, uint8_t *iso);

/* Per-kernel-class timing with HIP events recorded around each launch on the
 * launch stream (off by default; adds a small overhead when on).
 * amg_set_kernel_timing takes a bit mask of kinds (bit k enables kind k; 0
 * disables).  While timing is on, pcg_solve launches its iterations
 * individually instead of replaying a graph.  kind is one of the AMG_KIND_* values; *ms is the summed
 * duration, *launches the count, *bytes the summed algorithmic HBM bytes of
 * those launches. */
enum {
  AMG_KIND_SPMV_F64 = 0,      /* outer CG product q = A p                        */
  AMG_KIND_SWEEP = 1,         /* one colour pass of the level-0 smoother         */
  AMG_KIND_RESTRICT = 2,      /* level-0 residual + restriction                  */
  AMG_KIND_PROLONG = 3,       /* level-0 prolongation                            */
  AMG_KIND_CG_VEC = 4,        /* CG vector updates and dot products              */
  AMG_KIND_COARSE_LEVELS = 5, /* every launch of levels >= 1                     */
  AMG_KIND_OTHER = 6,         /* level-0 fills and the smoother's first pass     *
                               * from a zero iterate (x = b / diag)             */
  AMG_KIND_COUNT = 7
};
AMG_API amg_status amg_set_kernel_timing(int32_t kind_mask);
AMG_API amg_status amg_get_kernel_timing(int32_t kind, double *ms, int64_t *launches, double *bytes);
AMG_API amg_status amg_reset_kernel_timing(void);

#ifdef __cplusplus
}
#endif
#endif /* AMG_MI355X_AMG_H */
