/*
 * fiedler.h -- C ABI of the MI355X (gfx950) Fiedler-vector library: the
 * Gauss-Seidel cascadic multigrid method (GS-CMG) of S. Gandhi, "Improvement of
 * the Cascadic Multigrid Algorithm with a Gauss Seidel Smoother to Efficiently
 * Compute the Fiedler Vector of a Graph Laplacian", arXiv 1602.04386 (2015).
 *
 * Problem (Section 3, Definitions 2.1 and 2.2, and the text before Algorithm
 * 3): given the Laplacian L of a weighted undirected graph -- L_ii the weighted
 * degree, L_ij = -w_ij -- return the eigenvector phi_2 of the second smallest
 * eigenvalue lambda_2 (the algebraic connectivity) and lambda_2 itself, taken
 * as the finest-level Rayleigh quotient.
 *
 * Conventions for every entry point:
 *  - Every function returns fv_status (or void for destructors); no C++
 *    exception crosses this boundary.
 *  - Sizes are int32 / int64 as declared; CSR indices are int32 with
 *    0 <= nnz <= INT32_MAX.
 *  - The caller owns every array it passes.  Inputs are copied (or only read
 *    during the call); nothing the caller passes is retained after return,
 *    except where fv_submit says otherwise.
 *  - A context is not thread-safe; use one per thread.  Server entry points
 *    (fv_submit, fv_poll) are thread-safe.
 *  - Work runs on the context's HIP stream (or the stream in fv_solve_opts);
 *    entry points return after the results are in the caller's buffers.
 */
#ifndef FIEDLER_H
#define FIEDLER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FV_OK = 0,
  FV_PENDING = 1,            /* fv_poll: request not finished yet */
  FV_E_INVALID = -1,         /* null pointer, n < 2, row_ptr not starting at 0 / not
                                non-decreasing / not ending at nnz, column out of range,
                                columns not strictly ascending in a row, bad option */
  FV_E_NOT_SYMMETRIC = -2,   /* entry (i,j) without a bitwise-equal entry (j,i) */
  FV_E_NOT_LAPLACIAN = -3,   /* non-finite value; off-diagonal weight not > 0; L input:
                                diagonal missing or |L_ii - sum_j w_ij| > 1e-12 max(1,|L_ii|);
                                adjacency input: a diagonal entry present */
  FV_E_ISOLATED = -4,        /* a vertex without edges: lambda_2 = 0, phi_2 not unique */
  FV_E_NOMEM = -5,           /* device allocation failed */
  FV_E_BUDGET = -6,          /* the request does not fit the HBM budget */
  FV_E_NOT_CONVERGED = -7,   /* tol_res not met, or the coarsest solve hit its cap;
                                x, lambda and stats are still filled */
  FV_E_DEVICE = -8,          /* HIP runtime error */
  FV_E_UNKNOWN_TICKET = -9,  /* fv_poll: ticket never issued or already collected */
  FV_E_BUSY = -10,           /* server queue full */
  FV_E_SCRATCH = -11         /* fv_fiedler_solve_noalloc: the graph needs more than the
                                fixed scratch of FV_NOALLOC_SCRATCH_BYTES */
} fv_status;

typedef enum {
  FV_PREC_FP64 = 0,       /* every vector and weight in FP64 */
  FV_PREC_FP32_MIXED = 1  /* vectors and weights stored in FP32 for smoothing,
                             power iteration and prolongation (half the bytes);
                             reductions, shifts, projection, normalisation, the
                             coarsest solve and the final Rayleigh quotient and
                             residual (with FP64 weights) stay FP64 */
} fv_precision;

#define FV_MAX_LEVELS 64
#define FV_SCHEDULE_CAP 1024

typedef struct fv_context fv_context;
typedef struct fv_hierarchy fv_hierarchy;
typedef struct fv_server fv_server;

/* A graph in CSR form.  is_adjacency = 0: the Laplacian L of Definition 2.1
 * (diagonal present).  is_adjacency = 1: the weights W (no diagonal).  Columns
 * must be strictly ascending inside each row and the matrix bitwise symmetric.
 * on_device = 1: the three arrays are device pointers (for example torch
 * tensors on the same GPU); 0: host pointers.  val is FP64. */
typedef struct {
  int32_t n;
  int32_t nnz;
  const int32_t* row_ptr; /* n + 1 */
  const int32_t* col;     /* nnz */
  const double* val;      /* nnz */
  int32_t is_adjacency;
  int32_t on_device;
} fv_csr;

/* Setup options (Algorithm 3, Step 1).  Coarsen while a level has more than
 * n_coarse vertices (the text asks for about 25), for at most max_levels
 * levels.  colour_seed seeds the smoother's colouring.  ell chooses the
 * storage the smoothing sweeps read: with 0, on a level of more than 8,192
 * rows whose longest row has at most 32 entries, each of the first 32 colours
 * also keeps a slot-major (ELL) block of its rows of the solve-order matrix,
 * every row padded to the level's longest rounded up to a multiple of 4 slots
 * (16 bytes per slot, counted in fv_hierarchy_bytes), when the padding adds at
 * most an eighth to the colour's entries or at most 8 MiB of FP32 index and
 * weight; the colour's sweep launches then read that block instead of the CSR
 * arrays.  -1 keeps CSR only.  The two give bitwise-equal solves. */
typedef struct {
  int32_t n_coarse;     /* default 25 */
  int32_t max_levels;   /* default and maximum FV_MAX_LEVELS */
  uint64_t colour_seed; /* default 0 */
  int32_t ell;          /* default 0 (ELL copies where they fit); -1: CSR only */
} fv_hier_opts;

/* Solve options (Algorithm 3, Steps 2 and 3; stopping rule of Section 4). */
typedef struct {
  int32_t prec;          /* fv_precision */
  uint64_t seed;         /* SplitMix64 seed of the coarsest random start */
  double tol_cos;        /* a phase ends when (x_k, x_{k-1}) > 1 - tol_cos; Section 4
                            uses 1e-6; <= 0: no cosine stop, every phase runs to its cap
                            (a test against exactly 1 would fire on rounding) */
  double tol_res;        /* > 0: repeat the finest-level phases until
                            ||L x - lambda x|| / ||x|| <= tol_res; 0 = off */
  double omega;          /* relaxation of the smoothing sweep; 1 = Gauss-Seidel */
  int32_t max_gs;        /* sweeps per smoothing phase */
  int32_t max_pi;        /* steps per power-iteration phase */
  int32_t max_outer;     /* finest-level repeats for tol_res */
  int32_t max_coarsest;  /* coarsest power-iteration steps */
  const int32_t* replay; /* NULL, or a host array with the exact phase counts to run
                            (layout of fv_solve_stats.schedule); for reproducing a
                            schedule step for step */
  int32_t replay_len;
  void* stream;          /* hipStream_t to run on, or NULL for the context's stream */
  double tol_coarse;     /* the coarsest power iteration (Algorithm 3, Step 2) stops
                            once ||L x - (x^T L x) x|| <= tol_coarse * sigma for the
                            unit iterate x; the paper leaves this tolerance open.
                            Default 1e-13 */
  int32_t time_finest;   /* 1: time every finest-level smoothing launch with a pair
                            of HIP events (totals in fv_solve_stats; the first 2048
                            launches of a solve); 0 (default): no timing */
  int32_t early_exit;    /* 1: end the finest rounds of tol_res once the residual,
                            falling each round by its last reduction factor
                            (residual / the previous round's residual, products
                            taken one round at a time in double), cannot reach
                            tol_res within the rounds max_outer leaves, or did not
                            fall; such a solve returns FV_E_NOT_CONVERGED early (a
                            serving policy, not part of Section 4's rule).
                            0 (default): rounds until tol_res or max_outer */
} fv_solve_opts;

/* Per-solve statistics.  schedule = [coarsest steps, then (gs sweeps, pi steps)
 * for levels J-1 down to 0, then (gs, pi) per extra finest-level round]. */
typedef struct {
  int32_t levels;
  int32_t n[FV_MAX_LEVELS];
  int64_t nnz[FV_MAX_LEVELS];
  int32_t colours[FV_MAX_LEVELS];
  int32_t schedule_len;
  int32_t schedule[FV_SCHEDULE_CAP];
  double lambda;
  double residual;   /* ||L x - lambda x|| / ||x|| with FP64 weights */
  double final_cos;
  double t_solve_ms; /* device time of the solve (HIP events) */
  int64_t alg_bytes; /* algorithmic HBM bytes of the refinement passes */
  /* with fv_solve_opts.time_finest: the finest-level smoothing launches that
     were timed, their summed event time and their algorithmic bytes (per
     launch: its colour's rows and entries, as in alg_bytes) */
  int32_t n_finest_gs;
  double t_finest_gs_ms;
  int64_t finest_gs_bytes;
} fv_solve_stats;

/* Fills opts with the defaults named above (FP64, seed 1, tol_cos 1e-6, no
 * tol_res, omega 1, 100 sweeps, 100 steps, 50 rounds, 100000 coarsest steps). */
void fv_hier_opts_default(fv_hier_opts* opts);
void fv_solve_opts_default(fv_solve_opts* opts);

/* Creates a context on HIP device `device`.  hbm_budget_bytes bounds the device
 * memory that hierarchies and solves of this context may hold (0 = no bound).
 * Errors: FV_E_INVALID (bad device, null out), FV_E_DEVICE. */
fv_status fv_context_create(int device, size_t hbm_budget_bytes, fv_context** out);
/* Every hierarchy and server made with ctx must be freed before this call. */
void fv_context_destroy(fv_context* ctx);

/* Setup phase (Algorithm 3, Step 1; Algorithm 1).  Validates the input
 * (errors as listed in fv_status), copies it to the device and builds the level
 * hierarchy there: heavy-edge matching under a strict total edge order
 * (weight, then a pair hash, then the indices), attachment of unmatched
 * vertices to their heaviest neighbour's aggregate, aggregates numbered by
 * smallest member, Galerkin coarse graphs I L I^T summed in a fixed order, a
 * first-fit colouring per level for the multicolour smoother, and the shift
 * 2 max_i d_i per level.  The hierarchy is device-resident until
 * fv_free_hierarchy.  Errors: input errors, FV_E_NOMEM, FV_E_BUDGET,
 * FV_E_DEVICE. */
fv_status fv_build_hierarchy(fv_context* ctx, const fv_csr* L, const fv_hier_opts* opts,
                             fv_hierarchy** out);

/* The setup phase of fv_build_hierarchy for many graphs at once (the batched
 * solve's inputs): `threads` host threads (<= 0: up to 8), each with its own
 * HIP stream, build graphs[0 .. count) concurrently, so the latency-bound
 * setup rounds of different graphs overlap on the device.  out[i] receives
 * graph i's hierarchy, exactly the one fv_build_hierarchy builds, or NULL
 * when its build failed; item_status[i] (may be NULL) its status.  Every
 * hierarchy is complete on the device when the call returns.  Returns FV_OK
 * when every graph was built, else the status of the first failed graph (in
 * index order); FV_E_INVALID for a NULL ctx, graphs or out, or count < 0. */
fv_status fv_build_hierarchies(fv_context* ctx, int32_t count, const fv_csr* const* graphs,
                               const fv_hier_opts* opts, int32_t threads, fv_hierarchy** out,
                               fv_status* item_status);

/* Level count and per-level sizes (arrays of FV_MAX_LEVELS entries, any may be
 * NULL): vertices, stored off-diagonal entries, colours, shift sigma. */
fv_status fv_hierarchy_info(const fv_hierarchy* h, int32_t* levels, int32_t* n, int64_t* nnz,
                            int32_t* colours, double* sigma);

/* Device bytes the hierarchy holds (counted against its context's HBM
 * budget while the hierarchy lives).  FV_E_INVALID for a NULL argument. */
fv_status fv_hierarchy_bytes(const fv_hierarchy* h, int64_t* bytes);

/* Slots per row of the ELL block of colour `colour` of level `level` (its
 * smoothing launches read it; fv_hier_opts.ell), 0 when that colour is swept
 * from CSR (colours count in solve order, as fv_hierarchy_export_level's
 * colour array numbers them).  FV_E_INVALID for a NULL argument or a level
 * out of range. */
fv_status fv_hierarchy_ell_width(const fv_hierarchy* h, int32_t level, int32_t colour,
                                 int32_t* width);

/* Copies level `level` to host buffers in the canonical numbering (vertices of
 * a coarse level numbered by their aggregate's smallest member): row_ptr[n+1],
 * col[nnz], w[nnz] (off-diagonal weights), q[n] (aggregate of each vertex in
 * the next level) and colour[n]; q and colour are left untouched on the
 * coarsest level.  Any pointer may be NULL. */
fv_status fv_hierarchy_export_level(const fv_hierarchy* h, int32_t level, int32_t* row_ptr,
                                    int32_t* col, double* w, int32_t* q, int32_t* colour);

void fv_free_hierarchy(fv_hierarchy* h);

/* Coarsest solve and cascadic refinement (Algorithm 3, Steps 2-3), then the
 * finest Rayleigh quotient.  Per level, coarse to fine: prolongation
 * x = I^T y (Step 3), a smoothing phase of multicolour Gauss-Seidel sweeps on
 * (L - rho I) x = 0 with rho the Rayleigh quotient of the current iterate
 * (Algorithm 2), then a power-iteration phase on sigma I - L; after every sweep
 * or step the iterate is projected against the all-ones vector and normalised
 * and the phase ends on the cosine test or its cap.  x_out (n doubles; device
 * pointer when x_on_device) receives phi_2, unit length, orthogonal to ones,
 * signed so that its first entry with |x_i| >= 1e-3 max|x| is positive.
 * lambda_out and stats may be NULL.  Errors: FV_E_INVALID, FV_E_NOMEM,
 * FV_E_BUDGET, FV_E_NOT_CONVERGED (results still written), FV_E_DEVICE. */
fv_status fv_fiedler_solve(fv_context* ctx, const fv_hierarchy* h, const fv_solve_opts* opts,
                           double* x_out, int32_t x_on_device, double* lambda_out,
                           fv_solve_stats* stats);

/* The same solve for `count` hierarchies in one persistent launch: one
 * workgroup owns one graph at a time and takes the next from a
 * largest-first queue.  x_out[k], lambda_out[k], stats[k] and item_status[k]
 * belong to h[k]; lambda_out, stats and item_status may be NULL.  opts applies
 * to every item (replay must be NULL).  Returns FV_OK when the launch ran; each
 * item's own status is in item_status. */
fv_status fv_fiedler_solve_batch(fv_context* ctx, int32_t count, const fv_hierarchy* const* h,
                                 const fv_solve_opts* opts, double* const* x_out,
                                 int32_t x_on_device, double* lambda_out, fv_solve_stats* stats,
                                 fv_status* item_status);

/* Bytes of the fixed device scratch behind fv_fiedler_solve_noalloc (per GPU,
 * held from the first use of the library on that GPU until the process ends).
 * It holds the solve's workspace: two vectors and one FP64 scratch vector of
 * the finest level's size (8 bytes per vertex each), the per-block partial
 * sums and the device state, so graphs of up to about 1.3 million vertices
 * fit. */
#define FV_NOALLOC_SCRATCH_BYTES (32u << 20)

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same solve as
 * fv_fiedler_solve -- same kernels, same arithmetic, bitwise the same results
 * -- with no device or host allocation.  Its workspace is the fixed scratch
 * above instead of context memory, and the context's host buffers and events
 * (made by fv_context_create) are reused; nothing is counted against the
 * context's HBM budget.  The hierarchy, opts and outputs are as for
 * fv_fiedler_solve (x_out on the host or, with x_on_device, on the device).
 * Every call on one GPU shares that GPU's scratch and the context's host
 * buffers: calls that overlap on one GPU (other threads, other contexts, other
 * streams) race and must be serialised by the caller.  The scratch keeps the
 * last call's contents; the solve clears what it needs.  opts->time_finest is
 * ignored (its events would be created on first use).  Errors: as
 * fv_fiedler_solve, plus FV_E_SCRATCH when the hierarchy's workspace exceeds
 * FV_NOALLOC_SCRATCH_BYTES (nothing runs). */
fv_status fv_fiedler_solve_noalloc(fv_context* ctx, const fv_hierarchy* h,
                                   const fv_solve_opts* opts, double* x_out,
                                   int32_t x_on_device, double* lambda_out,
                                   fv_solve_stats* stats);

/* Launch options of a batch (pattern of the persistent batched launch; not a
 * paper step).  The launch configuration is the dynamic LDS each workgroup
 * gets for a graph's level vector and staged CSRs, and with it the number of
 * resident workgroups; every configuration gives bitwise the same results.
 * fv_batch_opts_default: no autotuning, no capture, the default LDS. */
typedef struct {
  int32_t autotune;  /* 0: default configuration; 1: the autotuner's choice for
                        the batch's size class (median and largest finest level,
                        count, mean degree), found on the first call of a class
                        by timing each candidate LDS size on a sample of the
                        batch and cached for the process; 2: the cached choice
                        when there is one, never tuning */
  int32_t graph;     /* 1: capture the launch sequence (task upload, queue reset,
                        the persistent launch, read-backs) in a hipGraph, kept by
                        the context with its buffers and replayed when the next
                        call repeats the same hierarchies, outputs and options */
  int64_t lds_bytes; /* > 0: force this LDS per workgroup (bytes, at most 147456) */
  /* filled in by the call */
  int64_t lds_bytes_used;
  int32_t grid;      /* persistent workgroups launched */
  int32_t tuned;     /* the configuration came from the autotuner */
  int32_t replayed;  /* the launch replayed a captured graph */
  double launch_ms;  /* device time from the task upload to the last read-back */
} fv_batch_opts;

void fv_batch_opts_default(fv_batch_opts* opts);

/* fv_fiedler_solve_batch with launch options (NULL: the defaults); the
 * results are those of fv_fiedler_solve_batch, bit for bit.  A captured graph
 * holds its device buffers (counted against the HBM budget) until the next
 * captured call or fv_context_destroy. */
fv_status fv_fiedler_solve_batch_ex(fv_context* ctx, int32_t count,
                                    const fv_hierarchy* const* h, const fv_solve_opts* opts,
                                    fv_batch_opts* batch, double* const* x_out,
                                    int32_t x_on_device, double* lambda_out,
                                    fv_solve_stats* stats, fv_status* item_status);

/* ---- Spectral partitioning (the use of phi_2 the paper names: graph
 * partitioning and spectral clustering, Introduction and Conclusion) ---- */

typedef struct {
  int32_t parts; /* a power of two, >= 2: log2(parts) rounds of bisection */
  int32_t cut;   /* 0: median cut -- the smaller half by (phi_2 value, vertex
                    index) goes to the lower part; 1: sign cut -- phi_2 < 0 */
} fv_partition_opts;

typedef struct {
  int32_t parts;
  int32_t part_size_min, part_size_max;
  int32_t solves;        /* Fiedler solves run (one per part cut) */
  int32_t not_converged; /* of those, how many ended FV_E_NOT_CONVERGED (their
                            vector is still used) */
  double cut_weight;     /* total weight of the edges between parts */
  double total_weight;   /* total edge weight */
  double t_ms;           /* wall time of the call */
} fv_partition_stats;

/* Recursive spectral bisection: every part of the current round is cut in two
 * by its own Fiedler vector (its induced subgraph is extracted on the device,
 * a hierarchy built with hopts and solved with sopts), until `parts` parts.
 * Part p of a round becomes parts 2p and 2p + 1.  A vertex left without an
 * edge inside its part takes no part in that solve and joins the smaller half.
 * graph is the adjacency form (is_adjacency = 1); part_out receives n labels
 * in [0, parts) (device pointer when part_on_device).  Errors: input errors as
 * fv_build_hierarchy, FV_E_INVALID (parts not a power of two >= 2, the
 * Laplacian form), FV_E_NOMEM, FV_E_BUDGET, FV_E_DEVICE. */
fv_status fv_spectral_partition(fv_context* ctx, const fv_csr* graph,
                                const fv_hier_opts* hopts, const fv_solve_opts* sopts,
                                const fv_partition_opts* popts, int32_t* part_out,
                                int32_t part_on_device, fv_partition_stats* stats);

/* ---- Serving: continuous batching of Fiedler requests over one GPU ---- */

typedef struct {
  int32_t max_inflight;      /* requests on the device at once (slots) */
  int32_t queue_capacity;    /* pending requests before FV_E_BUSY */
  size_t hbm_budget_bytes;   /* device bytes for resident hierarchies plus in-flight work */
  int32_t cache_hierarchies; /* 1: keep hierarchies resident by graph_id (LRU) */
  fv_hier_opts hier;
  fv_solve_opts solve;       /* replay and stream must be NULL */
  int32_t workers;           /* worker threads, each with its own stream (0: 8; at most
                                max_inflight); with two or more, the first takes only
                                requests of up to 16384 vertices */
} fv_server_opts;

typedef struct {
  uint64_t graph_id;   /* cache key; used when the server caches hierarchies */
  const fv_csr* graph; /* read during fv_submit only when the graph is not cached;
                          the arrays must stay valid until fv_poll returns a final
                          status */
  double* x_out;       /* host buffer of n doubles; must stay valid until fv_poll
                          returns a final status */
} fv_request;

typedef struct {
  fv_status status;
  double lambda;
  double residual;
  double queue_ms;   /* submit -> start of device work */
  double latency_ms; /* submit -> completion */
  int32_t cache_hit;
  int64_t alg_bytes; /* algorithmic HBM bytes of the solve's refinement passes */
} fv_result;

fv_status fv_server_create(fv_context* ctx, const fv_server_opts* opts, fv_server** out);

/* Queues a request and returns its ticket.  Errors: FV_E_INVALID, FV_E_BUSY
 * (queue full), FV_E_BUDGET (the graph alone exceeds the budget). */
fv_status fv_submit(fv_server* s, const fv_request* req, uint64_t* ticket);

/* FV_PENDING while the request runs; otherwise fills *out and returns FV_OK,
 * after which the ticket is forgotten.  FV_E_UNKNOWN_TICKET for an unknown or
 * already collected ticket. */
fv_status fv_poll(fv_server* s, uint64_t ticket, fv_result* out);

/* Drains in-flight work, then frees the server and its cached hierarchies. */
void fv_server_destroy(fv_server* s);

const char* fv_status_str(fv_status st);

#ifdef __cplusplus
}
#endif

#endif /* FIEDLER_H */
