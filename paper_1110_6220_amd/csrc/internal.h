// Host-side internals shared by the C-ABI translation units (api.cpp,
// serve.cpp).  Not installed.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/eik.h"
#include "engine.h"

namespace eik {

extern thread_local std::string g_err;
int fail(int code, const char* fmt, ...);
double now_s();

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return ::eik::fail(EIK_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// A fixed region of device memory that buffers are carved from in order
// (the allocation-free entry point); `used` is reset by every call.
struct Bump {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  bool overflow = false;  // a buffer did not fit
};

// A device allocation that only grows.  With a graveyard, a buffer that
// grows keeps its old allocation there (freed later by the owner) instead of
// calling hipFree, which would wait for all work on the device.  With a bump
// region the buffer is carved from it instead and nothing is allocated.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  std::vector<void*>* graveyard = nullptr;
  uint64_t* gen = nullptr;  // bumped when the buffer moves (captured graphs go stale)
  Bump* bump = nullptr;
  hipError_t ensure(size_t need);
  void release();
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

// Buffers of one engine run.
struct Solver {
  DevBuf delta, st, visits, cell_inst, key, deps, ord, slot, head, tail, inflight, cursor, ctl, inst;
  DevBuf hblk, istat, iact, qgrp, queued;
  void release();
  std::vector<DevBuf*> bufs();
};

// A captured launch sequence of one problem set (graph replay): the graph
// and what the host needs after a replay.  Problem descriptors live in
// buffers of the plan; all other buffers it uses belong to the workspace and
// are re-initialised by the graph's own kernels on every replay.
struct Plan {
  uint64_t key = 0, gen = 0, last_use = 0;
  hipGraphExec_t pre = nullptr;   // preparation, coarse solve, ordering
  hipGraphExec_t post = nullptr;  // residual, statistics copy
  Engine e{};                     // the solver kernel's arguments ...
  int workers = 0, tile = 0;      // ... and launch shape (launched between events)
  DevBuf inst, cinst, cout;
  std::vector<Inst> host_inst;
  int64_t J = 0;
  std::vector<double> widths;  // band widths (empty: no bands)
  bool coarse_engine = false, want_resid = false;
};

// Per-device workspace, reused by every call on that device.
struct Workspace {
  std::mutex mu;
  Solver fine, coarse;
  DevBuf F, u, mask, src, q;          // staging of host inputs
  DevBuf cF, cmask, cq, cu, cout;     // coarse problems
  DevBuf crank, fmm_spill;            // coarse Fast Marching (FMSM)
  DevBuf sweep_stat, sweep_dirty;     // whole-grid sweeping
  DevBuf grid3;                       // 3-D solver: cell marks, round lists, counters
  DevBuf fmsm3;                       // 3-D FMSM: coarse grid, ranks, levels
  DevBuf F64, u64;                    // FP64 re-solve of FP32 problems
  DevBuf ready_at, trace, trace_n;    // diagnostic trace (EIK_TRACE)
  DevBuf wall_in, wall_cnt;           // wall density of masked problems
  std::vector<void*> graveyard;       // outgrown buffers (deferred frees)
  uint64_t gen = 1;                   // changes whenever a buffer moves
  std::vector<std::unique_ptr<Plan>> plans;  // captured graphs (eik_opts.graph)
  hipStream_t capture = nullptr;      // private stream for graph capture
  uint64_t uses = 0;
  bool defer_free = false;            // grow without hipFree (serving lanes)
  Ctl* ctl_host = nullptr;            // pinned: fine and coarse control blocks
  int32_t* host3 = nullptr;           // pinned: 3-D solver read-back (64 bytes)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // null: the solver kernel is not timed
  Bump* bump = nullptr;               // carve every buffer from here (no allocation)
  int cus = 0;
  int wall_khz = 0;
  bool ready = false;
};

struct Tiling {
  int s, kx, ky, balanced, extent;
};

struct RunInfo {
  float kernel_ms;
  int64_t cells;
};

// The calling device's shared workspace (created on first use).
int workspace(Workspace** out);
// Initialises a workspace for the current device (pinned control block,
// events, device attributes; with a bump region only the device attributes:
// the caller provides ctl_host, and no event is created).
int workspace_init(Workspace* w);
// Frees everything a workspace holds (no work may be pending on it).
void workspace_free(Workspace* w);
// Makes the workspace's buffers grow without calling hipFree.
void workspace_defer_frees(Workspace* w);
// Share of accessible nodes next to an obstacle (host mask, sampled rows).
double wall_density_host(const eik_problem& p);

// Where a run takes its buffers from.  Defaults: the device's shared
// workspace for everything.
struct RunCtx {
  Workspace* ws = nullptr;       // workspace (and its lock) of this run
  void* const* delta = nullptr;  // per problem: nodes x dtype for h/F
  void* const* f64 = nullptr;    // per problem: 3 x nodes doubles (F, u, delta)
                                 // for the FP64 re-solve of FP32 problems
  int share = 1;                 // the run gets 1/share of the default waves
  const double* density = nullptr;  // per problem: wall density, if known
  // early completion: per problem a host-visible flag the solver sets when
  // that problem is solved (idone, zeroed by the caller), and a function
  // called repeatedly while the solver runs; problems whose results the
  // caller has taken (detached[k] != 0) get no FP64 re-solve afterwards
  unsigned int* idone = nullptr;
  std::function<void(const Engine&, const std::vector<Inst>&)> poll;
  const char* detached = nullptr;
};
// Band width of the band schedule: `width` if > 0, else `cells` times the
// problem's cell crossing at unit speed (s h).
struct BandSpec {
  double width, cells;
  double width_of(const Inst& I) const { return width > 0.0 ? width : cells * I.s * I.h; }
};
// Sizes the solver's buffers for the instances in `inst` (cell0 filled in)
// and fills the engine arguments.  band: the band schedule's widths, or
// nullptr (no bands).
int setup_engine(Solver& sv, std::vector<Inst>& inst, int dtype, int method, int dag, int heap,
                 const BandSpec* band, int window, int eager, uint64_t guard, uint64_t timeout,
                 hipStream_t stream, Engine* out, DevBuf* instbuf = nullptr, int rings = 1);
eik_opts default_opts();
int check_opts(const eik_opts& o);
int std_cells(int n, int s);
int make_tiling(int nx, int ny, int s, int method, Tiling* t);
int default_cell(int nx, int ny, int method);
size_t dsize(int dtype);
int validate_host(const eik_problem& p, int dtype);
int validate_shape(const eik_problem& p);
int validate_device(const eik_problem& p, int dtype);
// Solves n problems (validated) with one persistent launch.
int run(int n, const eik_problem* probs, const eik_opts& o, eik_stats* stats, RunInfo* info,
        const RunCtx* ctx = nullptr);
// Re-solves the FP32 problems probs[which[x]] in FP64 (device buffers of
// inst[which[x]]) and rounds the results into their FP32 outputs; resid[x]
// receives each FP64 solution's residual.
int refine_fp64(const std::vector<int>& which, const eik_problem* probs,
                const std::vector<Inst>& inst, const eik_opts& o, hipStream_t stream,
                const RunCtx& ctx, std::vector<double>* resid);

}  // namespace eik
