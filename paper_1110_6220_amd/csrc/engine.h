// Internal interface between the C-ABI layer (api.cpp) and the HIP engine
// (engine.hip).  Not installed; the public interface is include/eik.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eik {

// Per-cell state word.  kPending: queued or to be processed again; kRunning:
// a wave is processing the cell; kDone1: its first processing has finished
// (cells that are not ordered by dependency counts start with kDone1 set).
// Bits 8..11: preferred sweep directions raised by neighbours (0 SW, 1 NW,
// 2 NE, 3 SE); bits 12..15: the sides (0 W, 1 E, 2 S, 3 N) those neighbours
// sit on.
constexpr uint32_t kPending = 1u;
constexpr uint32_t kRunning = 2u;
constexpr uint32_t kDone1 = 4u;
constexpr int kFlagShift = 8;
constexpr int kSideShift = 12;

// Per-cell order bits (DAG ordering): bits 0..3 = sides (0 W, 1 E, 2 S, 3 N)
// whose neighbour comes earlier in the coarse order; kOrdConverge = the cell
// holds exit nodes or the coarse front never reaches it (FMSM sweeps it to
// convergence); kOrdEmpty = the cell has no accessible node.
constexpr uint8_t kOrdConverge = 0x10;
constexpr uint8_t kOrdEmpty = 0x20;
constexpr uint8_t kOrdSource = 0x40;  // the cell holds exit nodes

enum Method : int32_t { kExact = 0, kFmsm = 1, kFhcm = 2 };

// One problem instance.  Cell k along an axis of n nodes with K cells covers
// [lo(k), lo(k+1)) where lo(k) = k*s (and lo(K) = n) for the standard tiling,
// or floor(k*n/K) for the balanced one.
struct Inst {
  void* u;               // solution / working values (dtype)
  const void* F;         // speed (dtype; coarse problems: double)
  const uint8_t* mask;   // 1 accessible, 0 obstacle; nullptr = all accessible
  void* delta;           // workspace: h/F; +inf on obstacles and exit nodes (dtype)
  const int64_t* src;    // exit nodes (nsrc entries) ...
  const double* q;       // ... and their costs (nullptr = 0)
  const double* qdense;  // or: exit cost per node, +inf elsewhere (coarse problems)
  double h;
  int32_t nx, ny;
  int32_t s;             // nominal cell side
  int32_t kx, ky;        // cells per axis
  int32_t balanced;      // tiling kind
  int32_t cell0;         // global id of the instance's first cell
  int32_t nsrc;
};

// One problem's bands when a batch runs under the band schedule: each
// problem has its own rings, cursor and band width, so no problem waits for
// another's band to drain.
struct QGroup {
  unsigned long long off;  // first slot of the group's nb rings
  uint32_t cap;            // power of two > the problem's cells
  uint32_t pad;
  double inv_width;        // 1 / band width
  double pad2;
};

// Multi-producer multi-consumer cell queue.  Band b holds a ring of `cap`
// slots; a slot is (sequence << 32 | cell).  Keys map to absolute band index
// floor(key / width); the ring is that index modulo nb.  inflight[b] counts
// the cells of band b that are queued or running; the cursor moves past a
// band only once its count is zero (the band is closed with kClosed while the
// cursor moves, then reopened for band + nb).  Cells are popped only from the
// `window` + 1 bands starting at the cursor.  nb = 1 is a FIFO, for batches
// split into nring rings (no more rings than waves) so that the pushes and
// pops of many waves do not all meet on one head and one tail: a cell goes
// to ring (cell mod nring), a wave waits on ring (its workgroup index mod
// nring).
// With ng > 1 groups (one per problem of a batch) every group is such a
// queue of its own: counters of ring r of group g at index g * nb + r, the
// cursor of group g at g * kCtrStride, slots and width from grp[g] (filled by
// the preparation kernel: width `width` if > 0, else width_cells times the
// problem's s h).
struct Queue {
  unsigned long long* slot;      // nb * cap (ng > 1: sum over groups of nb * cap)
  unsigned long long* head;      // ng * nb entries, stride kCtrStride
  unsigned long long* tail;      // ng * nb entries, stride kCtrStride
  unsigned long long* inflight;  // ng * nb entries, stride kCtrStride
  unsigned long long* cursor;    // ng entries, stride kCtrStride
  unsigned long long* queued;    // ng > 1: per group the cells pushed and not yet
                                 // popped (a hint for the scan), stride kCtrStride
  QGroup* grp;                   // ng entries (ng > 1)
  uint32_t cap;                  // power of two > number of cells (ng = 1)
  uint32_t nb;                   // power of two
  uint32_t window;
  uint32_t ng;                   // groups (1: one queue for all cells)
  double inv_width;              // 1 / band width (ng = 1)
  unsigned long long nslot;      // slots in all
  double width, width_cells;     // band width of the groups (see above)
  uint32_t nring;                // nb = 1: FIFO rings, a power of two (cell g in
                                 // ring g mod nring, each of `cap` slots at
                                 // slot + r * cap)
  uint32_t pad_r;
};
constexpr int kCtrStride = 16;  // 128 bytes between hot counters
constexpr uint32_t kFifoRings = 8;  // rings of the FIFO queue
constexpr unsigned long long kClosed = 1ull << 62;

// Device control block.  Counters that many waves update while cells are
// processed sit on cache lines of their own.
struct Ctl {
  unsigned long long active;      // cells waiting, queued or running
  unsigned long long pad_a[15];
  unsigned long long visits;      // cell removals (checked against guard)
  unsigned long long pad_v[15];
  unsigned long long guard;       // limit on total visits
  unsigned long long deadline;    // wall_clock64() value after which workers stop
  unsigned int err;               // kErr* bits
  unsigned int pad0;
  unsigned long long pad_g[13];
  // statistics, flushed once per wave when it exits
  unsigned long long sweeps;      // productive sweeps
  unsigned long long checks;      // convergence tests (no-change sweeps, tile checks)
  unsigned long long band_steps;  // cursor advances
  unsigned long long mon_checks;
  unsigned long long mon_ok;
  // phase timers (wall-clock ticks summed over waves), when profiling
  unsigned long long t_idle, t_claim, t_load, t_sweep, t_publish, t_finish;
  unsigned long long pad_s[5];
};
constexpr unsigned kErrSpeed = 1u, kErrSource = 2u, kErrGuard = 4u, kErrDeadline = 8u;

// Arguments of the engine kernels.
struct Engine {
  Inst* inst;            // device array of ninst descriptors
  Inst one;              // copy of inst[0], used when args_inst is set
  int32_t args_inst;     // the single descriptor is known on the host
  int32_t ninst;
  int32_t ncells;        // total cells J
  int32_t method;
  int32_t dtype;         // 0 f64, 1 f32
  int32_t dag;           // cells start when their earlier neighbours are done
  uint32_t* st;          // J state words
  uint32_t* visits;      // J removal counts
  int32_t* cell_inst;    // J instance ids (ninst > 1)
  unsigned long long* key;  // J orderable bits of the cell value (key_bits of a double)
  int32_t* deps;         // J unfinished earlier neighbours (dag)
  uint8_t* ord;          // J order bits (dag)
  Queue q;
  Ctl* ctl;
  // heap schedule: one wave processes cells one at a time in increasing
  // (cell value, cell index) order; hblk[b] = smallest key of the pending
  // cells 64 b .. 64 b + 63 (kKeyNone: none)
  int32_t heap;
  unsigned long long* hblk;
  // per instance k: istat[4k] visits, [4k+1] productive sweeps, [4k+2]
  // no-change sweeps (batches only), [4k+3] bits of the FP64 residual
  unsigned long long* istat;
  // early completion (null when off): iact[k] = cells of instance k waiting,
  // queued or running; when it drops to zero the instance is solved and
  // idone[k] (host-visible memory) is set to 1 with system-scope release
  unsigned long long* iact;
  unsigned int* idone;
  int32_t eager;         // publish after every productive sweep
  int32_t profile;       // accumulate phase timers in Ctl
  // diagnostic trace (null when off): per cell the wall clock when it was
  // last made ready; per visit {cell, ready, popped, loaded, swept, done}
  unsigned long long* ready_at;
  unsigned long long* trace;
  unsigned int* trace_n;
  unsigned int trace_cap;
  unsigned long long guard;          // limit on total cell visits
  int32_t guard_given;               // 1: guard was set by the caller (batches:
                                     // each problem gets its share of it), 0:
                                     // default (each problem 64 J_k + 1024)
  unsigned long long timeout_ticks;  // wall_clock64 ticks before workers give up
};

// Coarse grid of one fine instance (FMSM Part I): one node per cell.
struct CoarseOut {
  double* F;        // J mean speed over accessible nodes
  uint8_t* mask;    // J 1 = the cell has an accessible node
  double* q;        // J min exit cost over the cell's exit nodes, +inf if none
  double* u;        // J coarse solution (filled by the coarse solve)
  int32_t* rank;    // J acceptance rank of Fast Marching (FMSM), else nullptr
};

// Workspace of the coarse Fast Marching kernel for problems whose coarse grid
// does not fit in LDS (J entries per problem at the problem's cell0).
struct FmmSpill {
  double* delta;  // h^c / F^c, +inf on coarse obstacles
  double* fval;   // front values
  int32_t* st;    // -2 obstacle, -1 far, -3 accepted, else the front slot
  int32_t* fidx;  // front cells
};

// Host-side launchers (engine.hip).  All work is enqueued on `stream`.
// prepare: cell states, queue, delta, validation, u = +inf / exit costs, and
// (unless dag) the exit cells queued.
hipError_t launch_prepare(const Engine& e, int64_t max_nodes, hipStream_t stream);
hipError_t launch_solve(const Engine& e, int workers, int tile, hipStream_t stream);
// Solver waves that fit on one compute unit at once (registers and LDS).
int solve_waves_per_cu(int dtype, int method, int tile);
// FP64 residual of instances [inst0, inst0 + count) (count 0: all) into istat
hipError_t launch_residual(const Engine& e, int64_t max_nodes, hipStream_t stream, int inst0 = 0,
                           int count = 0);
// coarse speeds, masks and exit costs of every fine cell (cells of instance k
// at co[k].*[cell - cell0])
hipError_t launch_coarse_inputs(const Engine& fine, const CoarseOut* co_dev, int max_cells,
                                hipStream_t stream);
// Exact solve of every problem's coarse grid (values into co[k].u) when no
// problem has more than kCoarseJacobiMax coarse cells (one workgroup of up
// to 1024 threads per problem, up to kCoarseJacobiPer cells per thread);
// max_cells = the largest count.
constexpr int kCoarseJacobiPer = 8;
constexpr int kCoarseJacobiMax = 1024 * kCoarseJacobiPer;
hipError_t launch_coarse_jacobi(const Engine& fine, const CoarseOut* co_dev, int max_cells,
                                hipStream_t stream);
// Fast Marching on the coarse grid of every problem (FMSM Part I): values
// into co[k].u, acceptance ranks into co[k].rank.  Problems with at most
// lds_cells coarse cells work in LDS (kFmmLdsBytesPerCell bytes per cell),
// the others in `spill`.
constexpr int kFmmLdsBytesPerCell = 20;
hipError_t launch_coarse_fmm(const Engine& fine, const CoarseOut* co_dev, int lds_cells,
                             const FmmSpill& spill, hipStream_t stream);
// Whole-grid sweeping: tiles of kSweepTile x kSweepTile nodes (standard
// tiling, Inst.s = kSweepTile).  One launch sweeps the tiles of anti-diagonal
// `diag` (in the sweep's own order) of ordering `dir`; `tiles` = their count.
constexpr int kSweepTile = 64;
struct SweepArgs {
  unsigned long long* stat;  // this sweep: [0] largest decrease (bits of a
                             // non-negative double), [1] nodes decreased,
                             // [2] tiles swept, [3] tiles skipped
  uint8_t* dirty;            // per tile (locking): 1 = may change
  int32_t dir, diag, locking, pad;
};
hipError_t launch_sweep_diag(const Engine& e, const SweepArgs& a, int tiles, hipStream_t stream);
// locking: marks the tiles holding exit nodes and their neighbours
hipError_t launch_sweep_seed(const Engine& e, int nsrc, uint8_t* dirty, hipStream_t stream);
// Largest coarse grid the Fast Marching kernel keeps in LDS on this device.
int coarse_fmm_lds_cells();
// dependency counts and order bits from the coarse solutions; queues the
// cells that have no earlier neighbour
hipError_t launch_dag(const Engine& fine, const CoarseOut* co_dev, int max_cells,
                      hipStream_t stream);
// wall density of masked problems (cell-size tuning): counts must hold 2 n
// zeroed entries
struct WallIn {
  const uint8_t* mask;
  int32_t nx, ny;
};
hipError_t launch_wall_density(const WallIn* in_dev, int n, int64_t max_nodes,
                               unsigned long long* counts, hipStream_t stream);
// one wave sweeping one tile `sweeps` times: wall-clock ticks into ticks[0]
// (bits 0..62; side 32 or 64)
hipError_t launch_probe_sweep(int dtype, int side, int sweeps, unsigned long long* ticks,
                              hipStream_t stream);
// element-wise copies between precisions (FP32 results re-solved in FP64)
hipError_t launch_convert(const void* src, int src_dtype, void* dst, int dst_dtype, int64_t n,
                          hipStream_t stream);

}  // namespace eik
