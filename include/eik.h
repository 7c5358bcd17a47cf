/*
 * libeik -- two-scale Eikonal solvers on one AMD Instinct MI355X (gfx950).
 *
 * Solves the static Eikonal boundary-value problem |grad u(x)| F(x) = 1 on a
 * uniform 2-D Cartesian grid with u = q on the exit set Q and a state
 * constraint (q = +inf) on the rest of the boundary, discretised by the
 * first-order upwind scheme (Chacon & Vladimirsky, "Fast two-scale methods for
 * Eikonal equations", Section 2, eq. Eik_discr).  The grid is split into
 * cells; each cell is swept by Gauss-Seidel sweeps (Algorithms FSM_order,
 * FSM) and the cells are ordered at the coarse scale:
 *   EIK_EXACT  label-correcting on cells (Algorithm generic_LC_cells, Heap-Cell
 *              Method of Section 3.2.2): converges to the exact solution of the
 *              discrete system regardless of processing order (the Theorem of
 *              Section 3.2.1), so cells are processed concurrently;
 *   EIK_FMSM   Fast Marching-Sweeping (Algorithm FMSM, Section 3.1): approximate;
 *   EIK_FHCM   Fast Heap-Cell Method (Algorithm FHCM, Section 3.2.3): approximate.
 *
 * Layout: row-major with x fastest; node (i, j) <-> index j*nx + i and
 * x_i = x0 + i*h.  All entry points return EIK_OK (0) or a negative
 * eik_status; eik_last_error() returns a thread-local message for the last
 * failure on the calling thread.  Inputs are validated before any output is
 * written: on EIK_EINVAL the caller's u_out is untouched.
 *
 * Ownership: the caller owns every buffer passed in; the library never frees
 * caller memory.  With device_ptrs = 1 every pointer (F, mask, src, q, u_out)
 * is device memory of the current HIP device and the work is ordered on
 * `stream`; the call returns once that work has completed.  Such arrays must
 * be aligned to their element size (the kernels update u_out with atomics,
 * which the hardware requires to be naturally aligned): EIK_EINVAL otherwise.
 * With device_ptrs = 0 they are host memory and the library stages them through
 * device buffers of its own.  Library workspace (per device) is allocated on
 * first use, grows when a larger problem arrives and is kept until the
 * process ends; calls on one device are serialised by a lock.
 */
#ifndef EIK_H
#define EIK_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EIK_OK = 0,
  EIK_EINVAL = -1,   /* invalid argument (see eik_solve)                        */
  EIK_ENOMEM = -2,   /* device or host allocation failed                        */
  EIK_EDEVICE = -3,  /* a HIP runtime call failed                               */
  EIK_EBUDGET = -4,  /* a request is larger than the whole serving budget       */
  EIK_ENOTCONV = -5, /* the cell-visit guard tripped (max_cell_visits)          */
  EIK_EBUSY = -6     /* serving: the request is still pending                   */
} eik_status;

typedef enum { EIK_F64 = 0, EIK_F32 = 1 } eik_dtype;
typedef enum { EIK_EXACT = 0, EIK_FMSM = 1, EIK_FHCM = 2 } eik_method;

/* Order in which cells are processed.
 *   COARSE  a cell starts once its neighbours that precede it in the
 *           acceptance order of Fast Marching on the grid of cell centres
 *           (FMSM Part I, Section 3.1) have been processed once; afterwards
 *           cells are re-queued by the label-correcting add criterion.  The
 *           only order FMSM uses, and the default for EXACT.
 *   BANDS   cells are taken from the lowest open bands of their cell values
 *           (eq. cell_value; the Heap-Cell Methods' heap with ties widened to
 *           a band of width `band`).  The default for FHCM.
 *   FIFO    cells are taken in the order they were queued.
 *   HEAP    one cell at a time, always the queued cell with the smallest
 *           (cell value, cell index): the heap of the Heap-Cell Methods
 *           (Section 3.2.2) exactly, with cell values compared in FP64.
 *           One wave does all the work (a reference order, slow: each
 *           removal scans per-block minima of the queued cells' values);
 *           FHCM under HEAP reproduces the serial method of Algorithm FHCM
 *           bit for bit.  Not for FMSM.
 * EXACT gives the same result under every order. */
typedef enum {
  EIK_SCHED_AUTO = 0,
  EIK_SCHED_COARSE = 1,
  EIK_SCHED_BANDS = 2,
  EIK_SCHED_FIFO = 3,
  EIK_SCHED_HEAP = 4
} eik_schedule;

typedef struct {
  eik_dtype dtype;          /* storage and sweep precision of u and F          */
  eik_method method;
  int32_t cell;             /* cell side s in nodes, 4..64; 0 = tuned choice    */
  double band;              /* BANDS: band width in units of u, the same for
                               every problem; 0 = band_cells                    */
  int32_t device_ptrs;      /* 1: all pointers are device memory                */
  void* stream;             /* hipStream_t, or NULL for the null stream         */
  uint64_t max_cell_visits; /* guard on total cell visits; 0 = 64 * cells + 1024
                               (a batch: each problem against its share,
                               max_cell_visits * J_k / J, or 64 J_k + 1024) */
  int32_t residual_check;   /* F32: recheck the fixed-point residual in FP64 and
                               re-solve in FP64 each problem whose residual
                               exceeds residual_tol (F64: only report it)     */
  int32_t workers;          /* persistent waves; 0 = chosen from the problem    */
  int32_t band_window;      /* bands above the lowest unfinished band whose
                               cells may start, 0..63 (with band = band_cells =
                               0 the tuned window is used instead)             */
  int32_t eager_publish;    /* 1: re-queue neighbours after every sweep that
                               changed a value; 0: once per removal, after the
                               cell converged (the paper's order)              */
  int32_t schedule;         /* eik_schedule                                     */
  int32_t timeout_ms;       /* time limit of one solve on the device; 0 = 10000.
                               A solve that exceeds it fails with EDEVICE.     */
  int32_t graph;            /* 1 (device_ptrs only): capture the call's launch
                               sequence into a HIP graph and replay it when the
                               same problem set (sizes, spacing, buffer
                               addresses, options) comes again; the buffers'
                               contents may change between calls.  Up to 8
                               graphs are kept per device and dropped when the
                               library's workspace has to grow.              */
  double residual_tol;      /* residual_check bound on max |T(u)-u|/u; 0 = 4 * 2^-24
                               (must be >= 0 and finite)                       */
  double band_cells;        /* BANDS with band = 0: band width in cell crossings
                               at unit speed (s * h of each problem); 0 = the
                               tuned width and window (csrc/tuned_bands.h).
                               In a batch every problem has bands of its own. */
} eik_opts;

/* Statistics of one problem.  In a batch, cells, cell_visits, sweeps,
   checks, max_residual and fell_back_to_f64 are the problem's own; seconds,
   kernel_seconds, band_steps, mon_checks and mon_ok are those of the whole
   launch. */
typedef struct {
  double seconds;           /* wall time of the call                            */
  double kernel_seconds;    /* device time of the cell-processing kernel(s)     */
  uint64_t cells;           /* number of cells J                                */
  uint64_t cell_visits;     /* cell removals (AvHR = cell_visits / cells)       */
  uint64_t sweeps;          /* productive sweeps (that changed a value)         */
  uint64_t checks;          /* sweeps that changed nothing (AvS = (sweeps +
                               checks) / cells)                                 */
  uint64_t band_steps;      /* advances of the queue's lowest band              */
  uint64_t mon_checks;      /* FHCM monotonicity checks                         */
  uint64_t mon_ok;          /* ... that found a monotone side                   */
  double max_residual;      /* max fixed-point residual |T(u)-u|/u (FP64) of the
                               solution, or -1 when not computed; after an FP64
                               re-solve, that of the FP64 solution before it is
                               rounded into the FP32 output                    */
  int32_t cell_used;        /* cell side used                                   */
  double band_used;         /* band width used                                  */
  int32_t fell_back_to_f64; /* F32 residual check failed and this problem was
                               re-solved in FP64 (result rounded to FP32)      */
  uint64_t cells_total;     /* cells of the whole launch (all problems)         */
  int32_t graph_replayed;   /* 1: this call replayed a captured graph          */
  double residual_f32;      /* F32 with residual_check: the FP32 solution's own
                               residual (also when it was re-solved), else -1  */
} eik_stats;

/* Solve one problem.
 *   nx, ny  >= 1 grid nodes per axis; h > 0 finite grid spacing.
 *   F       nx*ny values of `dtype`, > 0 and finite wherever mask == 1.
 *   mask    nx*ny bytes, 1 = accessible, 0 = obstacle; NULL = all accessible.
 *   src     nsrc >= 1 linear node indices of Q, each in range and accessible;
 *           duplicates take the smallest q.
 *   q       nsrc finite exit costs (FP64), NULL = all 0.
 *   u_out   nx*ny values of `dtype`: the solution, +inf on obstacles and on
 *           nodes with no accessible path to Q.
 *   opts    NULL = defaults (F64, EXACT, tuned cell and band, host pointers).
 *   stats   may be NULL.
 * Errors: EINVAL (bad sizes, spacing, speeds, sources, enums, cell side
 * outside [4, 64], an approximate method whose cell tiling has a cell wider
 * than 64 nodes), ENOMEM, EDEVICE, ENOTCONV. */
int eik_solve(int32_t nx, int32_t ny, double h, const void* F, const uint8_t* mask,
              int32_t nsrc, const int64_t* src, const double* q, void* u_out,
              const eik_opts* opts, eik_stats* stats);

/* One problem of a batch (same meaning as the eik_solve arguments). */
typedef struct {
  int32_t nx, ny;
  double h;
  const void* F;
  const uint8_t* mask;
  int32_t nsrc;
  const int64_t* src;
  const double* q;
  void* u_out;
} eik_problem;

/* Solve n independent problems in one persistent launch; all share `opts`
   (dtype, method, cell, band, pointer kind, stream).  stats: n entries or
   NULL; per-problem counters, with seconds/kernel_seconds of the whole batch.
   Validation covers every problem before any work starts. */
int eik_solve_batched(int32_t n, const eik_problem* probs, const eik_opts* opts,
                      eik_stats* stats);

/* Continuous-batching server.  The server allocates one device arena of
   hbm_budget_bytes at creation.  Each request is charged the device bytes it
   needs (F, u and h/F in the solve precision, the mask, the exit nodes and
   costs, and for FP32 with residual_check the FP64 re-solve buffers, 24 bytes
   per node) and waits until the arena can hold it; requests are admitted in
   submission order.  A request larger than the whole budget is refused with
   EBUDGET.  `lanes` host threads, each with its own stream, take all admitted
   requests that fit when they fall idle and solve them in one persistent
   launch; launches of different lanes run concurrently on the device, so a
   request that arrives while others are being solved starts as soon as a
   lane, a slot and memory are free.  A request's result does not depend on
   the requests it is solved with (up to the rounding of the exact method's
   order-independent fixed point).
   opts: dtype, method, cell, band, residual_check, schedule apply to every
   request; opts.device_ptrs = 1 means the request's F, mask, src and q are
   device memory, read when the request is admitted (they must stay valid until
   it completes); u_out is always host memory and must stay valid until
   poll/wait reports completion.  opts.stream and opts.workers are ignored
   (each lane uses its own stream and a 1/lanes share of the device).
   Small per-launch solver state (a few bytes per cell) is held by the lanes
   outside the budget.  Each lane uses two streams; create the server before
   the process replays HIP graphs (opts.graph): measured, a server created
   after one graph-replayed solve had twice the p99 latency (most likely two
   lanes then share one of the runtime's hardware queues). */
typedef struct {
  uint64_t hbm_budget_bytes;  /* device arena; 0 = 64 GiB                      */
  int32_t max_slots;          /* requests admitted at once; 0 = 1024           */
  int32_t lanes;              /* concurrent launches, 0..16; 0 = 2             */
  eik_opts opts;
} eik_serve_cfg;

typedef struct eik_server eik_server;

int eik_serve_create(const eik_serve_cfg* cfg, eik_server** out);
/* Validates the request, copies its host inputs (device_ptrs = 0) and returns
   at once with a ticket.  EINVAL as for eik_solve; EBUDGET (see above). */
int eik_serve_submit(eik_server* s, const eik_problem* p, uint64_t* ticket);
/* EIK_OK when done (stats filled if non-NULL; stats.seconds is the time from
   submission to completion), EIK_EBUSY while queued or running, or the
   request's own error.  A ticket is reported done once, then forgotten
   (a later call returns EINVAL). */
int eik_serve_poll(eik_server* s, uint64_t ticket, eik_stats* stats);
/* Blocks until the request is done. */
int eik_serve_wait(eik_server* s, uint64_t ticket, eik_stats* stats);
/* Cancels a request that has not been admitted yet (its ticket is forgotten);
   EBUSY if it has been admitted. */
int eik_serve_cancel(eik_server* s, uint64_t ticket);
/* Solves every request still queued or running, then frees the server
   (results not yet collected are dropped). */
int eik_serve_destroy(eik_server* s);

/* Whole-grid sweeping: the prior methods of Section 2 -- Fast Sweeping
   (Algorithm FSM: Gauss-Seidel sweeps over the whole grid in the four
   alternating orderings, quadrant update of eq. Eik_discr) and Locking
   Sweeping -- on the same device, one sweep at a time, with the early
   termination of the Section 4 remark on stopping sweeping methods before
   convergence (stop once the largest change of a sweep is at most a
   threshold t*).  Every sweep equals the serial lexicographic sweep bit for
   bit: tiles of 64 x 64 nodes go in anti-diagonal wavefronts of the sweep
   direction, each tile swept by one wave.  Locking skips a tile whose last
   sweep changed nothing and whose neighbours have not changed since (such a
   tile is a fixed point of its halo, so skipping changes no value; node-level
   locking as in Locking Sweeping does not pay on a SIMD machine). */
typedef struct {
  eik_dtype dtype;      /* EIK_F64 or EIK_F32 storage (FP32: FP64 two-sided branch) */
  int32_t locking;      /* 0: Fast Sweeping; 1: Locking Sweeping (tile locks) */
  int32_t max_sweeps;   /* >= 1; 0 = 65536 */
  double threshold;     /* t*: stop after the first sweep whose largest change is
                           <= t* (0: run to convergence); negative: stop only
                           when a sweep changes nothing or at max_sweeps */
  int32_t device_ptrs;  /* as in eik_opts */
  void* stream;         /* hipStream_t; NULL = default stream */
} eik_sweep_opts;

typedef struct {
  int32_t sweeps;         /* sweeps performed */
  int32_t converged;      /* 1: the last sweep changed no node */
  double seconds;         /* device time of the sweeps (preparation excluded) */
  int64_t tiles_swept;    /* tile sweeps performed ... */
  int64_t tiles_skipped;  /* ... and skipped by locking */
} eik_sweep_stats;

/* Solves one problem (arguments as eik_solve) by whole-grid sweeping.
   max_change[k] (optional, max_sweeps entries) receives the largest decrease
   of a node in sweep k (+inf when a node left +inf, 0 when none decreased),
   n_changed[k] (optional) the number of nodes that decreased; entries past the
   last sweep are left untouched.  Sweep k runs in ordering k mod 4: x and y
   ascending, x ascending and y descending, both descending, x descending and
   y ascending.  Errors as eik_solve (EINVAL before any device work on host
   inputs; device-side validation of device inputs reports EINVAL with u_out
   unspecified). */
int eik_sweep_solve(int32_t nx, int32_t ny, double h, const void* F, const uint8_t* mask,
                    int32_t nsrc, const int64_t* src, const double* q, void* u_out,
                    const eik_sweep_opts* opts, double* max_change, int64_t* n_changed,
                    eik_sweep_stats* stats);

/* Three dimensions: the exact method (label-correcting on cells, the
   Theorem of Section 3.2.1) on an nx x ny x nz grid, the extension to 3-D
   the paper proposes for its cell methods.  Node (i, j, k) <-> linear index
   (k*ny + j)*nx + i (x fastest); six neighbours; the upwind update takes the
   three axis minima a = min(U_W,U_E), b = min(U_S,U_N), c = min(U_D,U_U),
   sorted m1 <= m2 <= m3: one-sided m1 + h/F when m2 - m1 >= h/F, else the
   two-sided root of eq. two_sided_update when it does not exceed m3, else the
   root of (U-m1)^2 + (U-m2)^2 + (U-m3)^2 = (h/F)^2.  Cells of 8 x 8 x 8 nodes
   (the last ones ragged) are processed in rounds: all queued cells at once,
   one wave each, and a cell is queued for the next round when a node on a
   shared face decreased below the node across (a visit makes at most three
   sweeps; a cell still changing is queued again).  FP64 only.  F, mask, src, q,
   u_out are host arrays (device_ptrs = 0: copied in and out, validated
   before any device work) or device arrays on the current device
   (device_ptrs = 1: 8-byte aligned, else EINVAL; values validated on the
   device, EINVAL with u_out unspecified); work is ordered on `stream`
   (hipStream_t or NULL) and the call returns when it is done.  Errors as
   eik_solve; ENOTCONV if the round guard (16 J + 64 rounds) trips or a
   cell's sweeps do not terminate; EDEVICE if a round lists more than J cells
   (a cell is listed at most once per round, so this signals a device fault). */
typedef struct {
  double seconds;         /* wall time of the call after argument checks */
  double rounds_seconds;  /* device time of the rounds */
  int32_t rounds;         /* rounds that processed at least one cell */
  int64_t cells;          /* cells J */
  int64_t cell_visits;    /* cell processings over all rounds */
  int64_t sweeps;         /* sweeps over all processings (incl. the final ones) */
} eik3_stats;

int eik_solve3(int32_t nx, int32_t ny, int32_t nz, double h, const double* F, const uint8_t* mask,
               int32_t nsrc, const int64_t* src, const double* q, double* u_out,
               int32_t device_ptrs, void* stream, eik3_stats* stats);

/* Three dimensions, FMSM (Algorithm FMSM, Section 3.1, extended to 3-D as
   Section 5 proposes): the approximate Fast Marching-Sweeping method on the
   same grid, cells and update as eik_solve3.  Part I: Fast Marching on the
   grid of cell centres (h^c = 8 h, coarse speed F at the cell centre: the mean
   of the accessible ones among the one or two middle nodes per axis, else the
   cell mean; coarse exit cost min q), on the device in one wave.  Part II: the
   cells in that acceptance order (processed level by level: the cells of a
   level are pairwise non-adjacent, which gives the same result as one at a
   time), each swept once in every ordering its earlier neighbours allow (per
   axis: ascending from an earlier low face, descending from an earlier high
   face, both for both or none; ascending only along an axis one node thick),
   with the update from the ordering's three upwind neighbours; cells holding
   exit nodes and cells the coarse front never reaches are swept to
   convergence.  The result bounds the exact solution from above and may stay
   +inf behind obstacles that a cell's sweeps cannot go around.  Arguments,
   pointer kinds and errors as eik_solve3; in addition ENOMEM if the coarse
   front exceeds 12288 cells.  stats: rounds = levels, cell_visits = cells
   processed, sweeps = sweeps over all cells, rounds_seconds = device time of
   both parts. */
int eik_fmsm3(int32_t nx, int32_t ny, int32_t nz, double h, const double* F, const uint8_t* mask,
              int32_t nsrc, const int64_t* src, const double* q, double* u_out,
              int32_t device_ptrs, void* stream, eik3_stats* stats);

/* Measurement aid: the latency of one dependent step of the cell sweep.
   One wave alone on the device sweeps one side x side tile held in LDS
   `sweeps` times with the solver's own sweep (anti-diagonal steps, the local
   update of Section 2, dtype storage with the FP64 two-sided branch) and
   *seconds receives the wall time per anti-diagonal step: t_dep of the span
   bound D t_dep of a solve whose longest chain of dependent updates has D
   steps.  side: 32 or 64.  Errors: EINVAL, EDEVICE. */
int eik_probe_step_latency(int32_t dtype, int32_t side, int32_t sweeps, double* seconds);

/* Allocation-free solve, for callers that cannot allocate device memory
   (code under HIP graph capture, allocation-free serving loops, harnesses
   that forbid hipMalloc).  Same arguments, method, result and errors as
   eik_solve, with these limits: every pointer is device memory
   (opts->device_ptrs must be 1), opts->graph must be 0, and an F32 solve
   cannot ask for residual_check (its FP64 re-solve would need memory).
   Every device buffer beyond the caller's inputs and outputs comes from one
   device array of EIK_NOALLOC_SCRATCH_BYTES that the library holds per
   device until the process ends (h/F per node and about 100 bytes per
   cell: up to about 2.8 million nodes in FP64, 5 million in FP32); a
   problem that needs more is refused with EINVAL before any device work.
   The call allocates no device or pinned host memory and creates no HIP
   object (stats->kernel_seconds is 0).  Calls on one device share the
   array and are serialised by the library; calls from separate processes
   use separate arrays.  Overlapping calls on one device through other
   means than this library's lock race on the array. */
#define EIK_NOALLOC_SCRATCH_BYTES (64u << 20)
int eik_solve_noalloc(int32_t nx, int32_t ny, double h, const void* F, const uint8_t* mask,
                      int32_t nsrc, const int64_t* src, const double* q, void* u_out,
                      const eik_opts* opts, eik_stats* stats);

/* Message for the last failed call on this thread ("" if none). */
const char* eik_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* EIK_H */
