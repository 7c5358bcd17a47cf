// C-ABI layer of libeik: argument validation, per-device workspace, staging of
// host buffers, launch sequencing and statistics.  Declarations and the
// contract of every entry point are in include/eik.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/eik.h"
#include "engine.h"
#include "internal.h"
#include "tuned_bands.h"
#include "tuned_cells.h"

namespace eik {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// EIK_PROFILE=1 makes the solver accumulate per-phase wall-clock ticks,
// reported on stderr after each call (a diagnostic, off by default; the
// device side is compiled in only when the library is built with
// -DEIK_PROFILING).
static const bool g_profile = [] {
  const char* v = std::getenv("EIK_PROFILE");
  return v && v[0] == '1';
}();
// EIK_TRACE=<file> records one line per cell visit of the main solve
// (cell, sweeps, checks, ready, popped, loaded, swept, done in wall-clock
// ticks, hardware id) into <file> after each call (a diagnostic).
static const char* g_trace = std::getenv("EIK_TRACE");

hipError_t DevBuf::ensure(size_t need) {
  if (need <= bytes) return hipSuccess;
  if (bump) {
    const size_t at = (bump->used + 255) / 256 * 256;
    if (at > bump->cap || need > bump->cap - at) {
      bump->overflow = true;
      return hipErrorOutOfMemory;
    }
    p = bump->base + at;
    bytes = need;
    bump->used = at + need;
    return hipSuccess;
  }
  if (p) {
    if (graveyard) graveyard->push_back(p);
    else (void)hipFree(p);
  }
  if (gen) ++*gen;
  p = nullptr;
  size_t b = std::max<size_t>(need, 256);
  if (graveyard) b = std::max(b, 2 * bytes);  // geometric growth: few outgrown buffers
  bytes = 0;
  hipError_t e = hipMalloc(&p, b);
  if (e == hipSuccess) bytes = b;
  return e;
}

void DevBuf::release() {
  if (p && !bump) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

std::vector<DevBuf*> Solver::bufs() {
  return {&delta, &st,   &visits,   &cell_inst, &key, &deps, &ord,  &slot,  &head,
          &tail,  &inflight, &cursor, &ctl,      &inst, &hblk, &istat, &iact, &qgrp, &queued};
}

void Solver::release() {
  for (DevBuf* b : bufs()) b->release();
}

static std::vector<DevBuf*> all_bufs(Workspace* w) {
  std::vector<DevBuf*> v;
  for (Solver* sv : {&w->fine, &w->coarse})
    for (DevBuf* b : sv->bufs()) v.push_back(b);
  for (DevBuf* b : {&w->F, &w->u, &w->mask, &w->src, &w->q, &w->cF, &w->cmask, &w->cq, &w->cu,
                    &w->cout, &w->crank, &w->fmm_spill, &w->sweep_stat, &w->sweep_dirty, &w->grid3, &w->fmsm3, &w->F64,
                    &w->u64, &w->ready_at, &w->trace,
                    &w->trace_n, &w->wall_in, &w->wall_cnt})
    v.push_back(b);
  return v;
}

// Makes every buffer of the workspace grow without hipFree.
void workspace_defer_frees(Workspace* w) {
  w->defer_free = true;
  for (DevBuf* b : all_bufs(w)) b->graveyard = &w->graveyard;
}

static void drop_plan(Plan* pl) {
  if (pl->pre) (void)hipGraphExecDestroy(pl->pre);
  if (pl->post) (void)hipGraphExecDestroy(pl->post);
  pl->pre = pl->post = nullptr;
  pl->inst.release();
  pl->cinst.release();
  pl->cout.release();
}

void workspace_free(Workspace* w) {
  for (auto& pl : w->plans) drop_plan(pl.get());
  w->plans.clear();
  if (w->capture) (void)hipStreamDestroy(w->capture);
  w->capture = nullptr;
  for (void* p : w->graveyard) (void)hipFree(p);
  w->graveyard.clear();
  for (DevBuf* b : all_bufs(w)) b->release();
  if (w->ctl_host) (void)hipHostFree(w->ctl_host);
  if (w->host3) (void)hipHostFree(w->host3);
  w->host3 = nullptr;
  if (w->ev0) (void)hipEventDestroy(w->ev0);
  if (w->ev1) (void)hipEventDestroy(w->ev1);
  w->ctl_host = nullptr;
  w->ev0 = w->ev1 = nullptr;
  w->ready = false;
}

static std::mutex g_ws_mu;
static std::vector<std::unique_ptr<Workspace>> g_ws;

int workspace_init(Workspace* w) {
  if (w->ready) return EIK_OK;
  for (DevBuf* b : all_bufs(w)) {
    b->gen = &w->gen;
    b->bump = w->bump;
  }
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (w->bump) {  // nothing is allocated: read-back into the caller's ctl_host
    HIP_TRY(hipDeviceGetAttribute(&w->cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipDeviceGetAttribute(&w->wall_khz, hipDeviceAttributeWallClockRate, dev));
    if (w->wall_khz <= 0) w->wall_khz = 100000;
    w->ready = true;
    return EIK_OK;
  }
  HIP_TRY(hipHostMalloc((void**)&w->ctl_host, 2 * sizeof(Ctl), hipHostMallocDefault));
  HIP_TRY(hipHostMalloc((void**)&w->host3, 16 * sizeof(int32_t), hipHostMallocDefault));
  HIP_TRY(hipEventCreate(&w->ev0));
  HIP_TRY(hipEventCreate(&w->ev1));
  HIP_TRY(hipDeviceGetAttribute(&w->cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIP_TRY(hipDeviceGetAttribute(&w->wall_khz, hipDeviceAttributeWallClockRate, dev));
  if (w->wall_khz <= 0) w->wall_khz = 100000;
  w->ready = true;
  return EIK_OK;
}

int workspace(Workspace** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_ws_mu);
  if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
  if (!g_ws[dev]) g_ws[dev].reset(new Workspace());
  Workspace* w = g_ws[dev].get();
  int rc = workspace_init(w);
  if (rc) return rc;
  *out = w;
  return EIK_OK;
}

// ---------------------------------------------------------------------------
// options, tiling
// ---------------------------------------------------------------------------

eik_opts default_opts() {
  eik_opts o;
  std::memset(&o, 0, sizeof o);
  o.dtype = EIK_F64;
  o.method = EIK_EXACT;
  return o;
}

int check_opts(const eik_opts& o) {
  if (o.dtype != EIK_F64 && o.dtype != EIK_F32) return fail(EIK_EINVAL, "unknown dtype %d", (int)o.dtype);
  if (o.method != EIK_EXACT && o.method != EIK_FMSM && o.method != EIK_FHCM)
    return fail(EIK_EINVAL, "unknown method %d", (int)o.method);
  if (o.cell != 0 && (o.cell < 4 || o.cell > 64))
    return fail(EIK_EINVAL, "cell side %d outside [4, 64]", (int)o.cell);
  if (!(o.band == o.band) || std::isinf(o.band)) return fail(EIK_EINVAL, "band must be finite");
  if (!(o.band_cells >= 0.0) || std::isinf(o.band_cells))
    return fail(EIK_EINVAL, "band_cells must be >= 0 and finite");
  if (o.workers < 0) return fail(EIK_EINVAL, "workers must be >= 0");
  if (o.band_window < 0 || o.band_window > 63) return fail(EIK_EINVAL, "band_window outside [0, 63]");
  if (o.timeout_ms < 0) return fail(EIK_EINVAL, "timeout_ms must be >= 0");
  if (o.schedule < EIK_SCHED_AUTO || o.schedule > EIK_SCHED_HEAP)
    return fail(EIK_EINVAL, "unknown schedule %d", (int)o.schedule);
  if (!(o.residual_tol >= 0.0) || std::isinf(o.residual_tol))
    return fail(EIK_EINVAL, "residual_tol must be >= 0 and finite");
  if (o.method == EIK_FMSM && o.schedule != EIK_SCHED_AUTO && o.schedule != EIK_SCHED_COARSE)
    return fail(EIK_EINVAL, "FMSM processes cells in the coarse order only");
  if (o.method == EIK_FHCM && o.schedule == EIK_SCHED_COARSE)
    return fail(EIK_EINVAL, "FHCM orders cells by their cell values");
  return EIK_OK;
}

int std_cells(int n, int s) {
  int K = (n + s - 1) / s;
  if (K > 1 && n % s == 1) K--;
  return K;
}

static int tile_for(int extent) { return extent <= 16 ? 16 : extent <= 32 ? 32 : 64; }

// Standard tiling: K = ceil(n/s) cells of s nodes, a last cell of one node
// merged into its predecessor.  The exact method, whose result does not
// depend on the tiling, uses the balanced tiling instead (K = ceil(n/s) cells
// of floor/ceil n/K nodes) whenever the merged last cell would need a larger
// tile than s (e.g. n = 1025, s = 32: 33 cells of 31 or 32 nodes instead of a
// 33-node last cell).  The approximate methods keep the standard tiling and
// accept cells of at most 64 nodes.
int make_tiling(int nx, int ny, int s, int method, Tiling* t) {
  t->s = s;
  t->kx = std_cells(nx, s);
  t->ky = std_cells(ny, s);
  int ex = std::max({std::min(s, nx), nx - (t->kx - 1) * s, std::min(s, ny), ny - (t->ky - 1) * s});
  t->balanced = 0;
  if (ex > 64 && method != EIK_EXACT)
    return fail(EIK_EINVAL, "cell side %d leaves a cell of %d nodes (> 64) for this method", s, ex);
  if (method == EIK_EXACT && (ex > 64 || tile_for(ex) > tile_for(std::min(s, 64)))) {
    t->kx = (nx + s - 1) / s;
    t->ky = (ny + s - 1) / s;
    t->balanced = 1;
    ex = std::max((nx + t->kx - 1) / t->kx, (ny + t->ky - 1) / t->ky);
  }
  t->extent = ex;
  return EIK_OK;
}

int default_cell(int nx, int ny, int method) {
  const int n = std::max(nx, ny);
  if (method != EIK_EXACT) {
    // approximate methods need the standard tiling within 64 nodes
    if (n >= 512 && (nx % 64 != 1) && (ny % 64 != 1)) return 64;
    return n >= 160 ? 32 : 16;
  }
  return n >= 512 ? 64 : n >= 160 ? 32 : 16;
}

// Cell side for the exact method from the tuned table (first matching row).
static int tuned_cell(int dtype, bool batched, int nx, int ny, double wall_density) {
  const int n = std::max(nx, ny);
  const int dense = wall_density >= kDenseWalls ? 1 : 0;
  for (const TunedCell& t : kTunedCells)
    if (t.dtype == dtype && t.batched == (batched ? 1 : 0) && t.dense == dense && n <= t.nmax)
      return t.cell;
  return default_cell(nx, ny, EIK_EXACT);
}

// Band width (in cell crossings s h at unit speed) and window of the band
// schedule from the tuned table.
static void tuned_band(int method, int dtype, bool batched, double* factor, int* window) {
  *factor = 1.0;
  *window = 0;
  for (const TunedBand& t : kTunedBands)
    if (t.method == method && t.dtype == dtype && t.batched == (batched ? 1 : 0)) {
      *factor = t.factor;
      *window = t.window;
      return;
    }
}

// Wall density of host masks: the share of accessible nodes with an
// inaccessible 4-neighbour, estimated on every fourth row.
double wall_density_host(const eik_problem& p) {
  if (!p.mask) return 0.0;
  uint64_t acc = 0, wall = 0;
  for (int j = 0; j < p.ny; j += 4) {
    const uint8_t* m = p.mask + (size_t)j * p.nx;
    for (int i = 0; i < p.nx; ++i) {
      if (!m[i]) continue;
      acc++;
      wall += (i > 0 && !m[i - 1]) || (i + 1 < p.nx && !m[i + 1]) || (j > 0 && !m[i - p.nx]) ||
              (j + 1 < p.ny && !m[i + p.nx]);
    }
  }
  return acc ? (double)wall / (double)acc : 0.0;
}

static uint32_t pow2_at_least(uint64_t v) {
  uint32_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

size_t dsize(int dtype) { return dtype == EIK_F64 ? sizeof(double) : sizeof(float); }

// Host-side validation of host-resident inputs.
int validate_host(const eik_problem& p, int dtype) {
  const size_t n = (size_t)p.nx * p.ny;
  for (size_t k = 0; k < n; ++k) {
    if (p.mask && !p.mask[k]) continue;
    const double f = dtype == EIK_F64 ? static_cast<const double*>(p.F)[k]
                                      : (double)static_cast<const float*>(p.F)[k];
    if (!(f > 0.0) || !std::isfinite(f))
      return fail(EIK_EINVAL, "speed F[%zu] = %g is not positive and finite", k, f);
  }
  for (int s = 0; s < p.nsrc; ++s) {
    const long long k = p.src[s];
    if (k < 0 || k >= (long long)n) return fail(EIK_EINVAL, "source %d index %lld out of range", s, k);
    if (p.mask && !p.mask[k]) return fail(EIK_EINVAL, "source %d lies on an obstacle", s);
    if (p.q && !std::isfinite(p.q[s])) return fail(EIK_EINVAL, "source %d has non-finite q", s);
  }
  return EIK_OK;
}

// Device-resident inputs are read and written in place, u_out with 64-bit
// (FP64) or 32-bit atomics, which the hardware requires to be naturally
// aligned: every array must sit on a multiple of its element size.
int validate_device(const eik_problem& p, int dtype) {
  const auto off = [](const void* q, size_t a) { return reinterpret_cast<uintptr_t>(q) % a != 0; };
  if (off(p.F, dsize(dtype)) || off(p.u_out, dsize(dtype)))
    return fail(EIK_EINVAL, "F and u_out must be aligned to their element size");
  if (off(p.src, sizeof(int64_t)) || (p.q && off(p.q, sizeof(double))))
    return fail(EIK_EINVAL, "src and q must be 8-byte aligned");
  return EIK_OK;
}

int validate_shape(const eik_problem& p) {
  if (p.nx < 1 || p.ny < 1) return fail(EIK_EINVAL, "grid %d x %d is empty", p.nx, p.ny);
  if ((long long)p.nx * p.ny > (1ll << 31) - 1) return fail(EIK_EINVAL, "grid too large");
  if (!(p.h > 0.0) || !std::isfinite(p.h)) return fail(EIK_EINVAL, "h = %g must be positive and finite", p.h);
  if (!p.F || !p.u_out) return fail(EIK_EINVAL, "F and u_out are required");
  if (p.nsrc < 1 || !p.src) return fail(EIK_EINVAL, "at least one source is required");
  return EIK_OK;
}

// ---------------------------------------------------------------------------
// engine set-up
// ---------------------------------------------------------------------------

// Sizes the solver's buffers for the instances in `inst` (cell0 filled in
// here) and fills the engine arguments.
int setup_engine(Solver& sv, std::vector<Inst>& inst, int dtype, int method, int dag, int heap,
                 const BandSpec* band, int window, int eager, uint64_t guard, uint64_t timeout,
                 hipStream_t stream, Engine* out, DevBuf* instbuf, int rings) {
  DevBuf& ib = instbuf ? *instbuf : sv.inst;
  int64_t J = 0;
  for (auto& I : inst) {
    I.cell0 = (int32_t)J;
    J += (int64_t)I.kx * I.ky;
  }
  if (J > (1ll << 30)) return fail(EIK_EINVAL, "too many cells");
  const int n = (int)inst.size();
  // bands: one queue of 64 bands; a batch gets a group of bands per problem
  // (16, or enough for the window)
  const bool groups = band && n > 1;
  const uint32_t nb = !band ? 1u : groups ? std::max<uint32_t>(16u, pow2_at_least((uint64_t)window + 2)) : 64u;
  // FIFO: `rings` rings (no more than the waves that wait on them), each
  // holding at most the cells g with g mod rings equal to its index
  uint32_t nring = 1;  // a power of two (cells map to rings by their low bits)
  while (nb == 1 && nring * 2 <= (uint32_t)std::min<int>(rings, (int)kFifoRings)) nring *= 2;
  const uint32_t cap = pow2_at_least((J + nring - 1) / nring + 1);
  const uint32_t ng = groups ? (uint32_t)n : 1u;
  const uint32_t nctr = std::max<uint32_t>(ng * nb, nring);
  uint64_t nslot = (uint64_t)cap * nb * nring;
  if (groups) {  // the preparation kernel lays the groups out the same way
    nslot = 0;
    for (int k = 0; k < n; ++k) nslot += (uint64_t)pow2_at_least((uint64_t)inst[k].kx * inst[k].ky + 1) * nb;
  }
  HIP_TRY(sv.st.ensure(J * sizeof(uint32_t)));
  HIP_TRY(sv.visits.ensure(J * sizeof(uint32_t)));
  HIP_TRY(sv.key.ensure(J * sizeof(unsigned long long)));
  HIP_TRY(sv.istat.ensure(4 * (size_t)n * sizeof(unsigned long long)));
  HIP_TRY(sv.iact.ensure((size_t)n * sizeof(unsigned long long)));
  HIP_TRY(sv.hblk.ensure(heap ? ((J + 63) / 64) * sizeof(unsigned long long) : 8));
  HIP_TRY(sv.cell_inst.ensure(n > 1 ? J * sizeof(int32_t) : 4));
  HIP_TRY(sv.deps.ensure(dag ? J * sizeof(int32_t) : 4));
  HIP_TRY(sv.ord.ensure(dag ? J : 4));
  HIP_TRY(sv.slot.ensure((size_t)nslot * sizeof(unsigned long long)));
  HIP_TRY(sv.head.ensure((size_t)nctr * kCtrStride * sizeof(unsigned long long)));
  HIP_TRY(sv.tail.ensure((size_t)nctr * kCtrStride * sizeof(unsigned long long)));
  HIP_TRY(sv.inflight.ensure((size_t)nctr * kCtrStride * sizeof(unsigned long long)));
  HIP_TRY(sv.cursor.ensure((size_t)ng * kCtrStride * sizeof(unsigned long long)));
  HIP_TRY(sv.queued.ensure((size_t)ng * kCtrStride * sizeof(unsigned long long)));
  HIP_TRY(sv.qgrp.ensure((size_t)ng * sizeof(QGroup)));
  HIP_TRY(sv.ctl.ensure(sizeof(Ctl)));
  HIP_TRY(ib.ensure(n * sizeof(Inst)));
  HIP_TRY(hipMemcpyAsync(ib.p, inst.data(), n * sizeof(Inst), hipMemcpyHostToDevice, stream));
  Engine& e = *out;
  std::memset(&e, 0, sizeof e);
  e.inst = ib.as<Inst>();
  e.one = inst[0];
  e.args_inst = n == 1;
  e.ninst = n;
  e.ncells = (int32_t)J;
  e.method = method;
  e.dtype = dtype;
  e.dag = dag;
  e.st = sv.st.as<uint32_t>();
  e.visits = sv.visits.as<uint32_t>();
  e.cell_inst = sv.cell_inst.as<int32_t>();
  e.key = sv.key.as<unsigned long long>();
  e.heap = heap;
  e.hblk = sv.hblk.as<unsigned long long>();
  e.istat = sv.istat.as<unsigned long long>();
  e.iact = sv.iact.as<unsigned long long>();
  e.idone = nullptr;
  e.deps = sv.deps.as<int32_t>();
  e.ord = sv.ord.as<uint8_t>();
  e.q.slot = sv.slot.as<unsigned long long>();
  e.q.head = sv.head.as<unsigned long long>();
  e.q.tail = sv.tail.as<unsigned long long>();
  e.q.inflight = sv.inflight.as<unsigned long long>();
  e.q.cursor = sv.cursor.as<unsigned long long>();
  e.q.queued = sv.queued.as<unsigned long long>();
  e.q.grp = sv.qgrp.as<QGroup>();
  e.q.cap = cap;
  e.q.nb = nb;
  e.q.window = (uint32_t)window;
  e.q.ng = ng;
  e.q.inv_width = band ? 1.0 / band->width_of(inst[0]) : 0.0;
  e.q.nslot = nslot;
  e.q.nring = nring;
  e.q.width = band ? band->width : 0.0;
  e.q.width_cells = band ? band->cells : 0.0;
  e.ctl = sv.ctl.as<Ctl>();
  e.eager = eager;
  e.profile = g_profile;
  e.guard = guard ? guard : 64ull * (uint64_t)J + 1024ull;
  e.guard_given = guard ? 1 : 0;
  e.timeout_ticks = timeout;
  return EIK_OK;
}

// Persistent workers: as many as fit on the device at once (at most one per
// cell).  A single problem is capped at J/16 workers, between 128 and 256:
// beyond that more workers only contend for the few ready cells of one
// front.  Measured (kernel us at 128 / 256 / 512 workers): 4097^2
// checkerboard with obstacles (4225 cells) 7309 / 6799 / 6961, 2049^2 maze
// (4225 cells) 15577 / 14311 / 14081, 2049^2 smooth speed (1089 cells)
// 2272 / 2271 / 2302, 1025^2 (289 cells) 1146 / 1149 / 1162.
static int default_workers(const Workspace* ws, int64_t J, int tile, int dtype, int method, int n) {
  static std::mutex mu;
  static int cache[2][3][3] = {};
  const int ti = tile <= 16 ? 0 : tile <= 32 ? 1 : 2;
  int per_cu;
  {
    std::lock_guard<std::mutex> lk(mu);
    int& c = cache[dtype][method][ti];
    if (!c) c = solve_waves_per_cu(dtype, method, tile);
    per_cu = c;
  }
  int64_t w = std::min<int64_t>(J, (int64_t)ws->cus * per_cu);
  if (n == 1) w = std::min<int64_t>(w, std::min<int64_t>(256, std::max<int64_t>(128, J / 16)));
  return (int)std::max<int64_t>(w, 1);
}

// ---------------------------------------------------------------------------
// the solve driver shared by eik_solve, eik_solve_batched and the server
// ---------------------------------------------------------------------------

constexpr unsigned kTraceCap = 1u << 20;  // trace records (EIK_TRACE)
// Cell side of the cell engine when it solves a coarse grid (more than
// kCoarseJacobiMax coarse cells) for the order of the exact method: 16-node
// cells let several waves share the coarse front (the 65 x 65 coarse grid of
// the 4097^2 checkerboard, before Jacobi took grids of that size: ~0.47 ms
// in one 64-node cell, 0.34 ms in 16-node cells, 0.07 ms more in 32 or 64).
#ifndef EIK_COARSE_ENGINE_CELL
#define EIK_COARSE_ENGINE_CELL 16
#endif
constexpr int kCoarseEngineCell = EIK_COARSE_ENGINE_CELL;
constexpr size_t kMaxPlans = 8;           // captured graphs kept per workspace

static int complete(Workspace* ws, int n, const eik_problem* probs, const eik_opts& o,
                    const RunCtx& ctx, const std::vector<Inst>& inst, int64_t J, const std::vector<double>& widths,
                    bool coarse_engine, bool want_resid, const unsigned long long* istat,
                    hipStream_t stream, double t0, eik_stats* stats, RunInfo* info,
                    std::unique_lock<std::mutex>& lk, bool replayed);

// Identity of a problem set for graph replay: every input that shapes the
// launch sequence (sizes, spacing, buffer addresses, options).  The contents
// of the buffers may change between replays.
static uint64_t plan_key(int n, const eik_problem* probs, const eik_opts& o, const RunCtx& ctx) {
  uint64_t hsh = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t b) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < b; ++i) hsh = (hsh ^ c[i]) * 1099511628211ull;
  };
  mix(&n, sizeof n);
  for (int k = 0; k < n; ++k) {
    const eik_problem& p = probs[k];
    mix(&p.nx, sizeof p.nx);
    mix(&p.ny, sizeof p.ny);
    mix(&p.h, sizeof p.h);
    mix(&p.F, sizeof p.F);
    mix(&p.mask, sizeof p.mask);
    mix(&p.nsrc, sizeof p.nsrc);
    mix(&p.src, sizeof p.src);
    mix(&p.q, sizeof p.q);
    mix(&p.u_out, sizeof p.u_out);
    if (ctx.delta) mix(&ctx.delta[k], sizeof(void*));
  }
  for (const int32_t v : {(int32_t)o.dtype, (int32_t)o.method, o.cell, o.workers, o.band_window,
                          o.eager_publish, o.schedule, o.residual_check, o.timeout_ms, ctx.share})
    mix(&v, sizeof v);
  mix(&o.band, sizeof o.band);
  mix(&o.band_cells, sizeof o.band_cells);
  mix(&o.max_cell_visits, sizeof o.max_cell_visits);
  return hsh;
}

int run(int n, const eik_problem* probs, const eik_opts& o, eik_stats* stats, RunInfo* info,
        const RunCtx* ctx_in) {
  const double t0 = now_s();
  RunCtx ctx = ctx_in ? *ctx_in : RunCtx();
  Workspace* ws = ctx.ws;
  int rc = ws ? workspace_init(ws) : workspace(&ws);
  if (rc) return rc;
  ctx.ws = ws;
  std::unique_lock<std::mutex> lk(ws->mu);
  if (ws->bump) {  // every buffer is carved afresh from the start of the region
    ws->bump->used = 0;
    ws->bump->overflow = false;
    for (DevBuf* b : all_bufs(ws)) {
      b->p = nullptr;
      b->bytes = 0;
    }
  }
  hipStream_t stream = static_cast<hipStream_t>(o.stream);
  const int dt = o.dtype;
  const size_t es = dsize(dt);
  const int method = o.method;
  int sched = o.schedule;
  if (sched == EIK_SCHED_AUTO) sched = method == EIK_FHCM ? EIK_SCHED_BANDS : EIK_SCHED_COARSE;
  const bool dag = sched == EIK_SCHED_COARSE;
  const bool heap = sched == EIK_SCHED_HEAP;
  const bool dev = o.device_ptrs != 0;
  const bool want_resid = o.residual_check != 0;

  // graph replay: a problem set seen before (same buffers, sizes and options)
  // runs its captured launch sequence
  const bool use_graph = o.graph && dev && !g_trace && !g_profile && !ws->bump && !ctx.idone;
  const uint64_t key = use_graph ? plan_key(n, probs, o, ctx) : 0;
  ws->uses++;
  if (use_graph) {
    for (size_t x = 0; x < ws->plans.size(); ++x) {  // drop graphs of moved buffers
      if (ws->plans[x]->gen == ws->gen) continue;
      drop_plan(ws->plans[x].get());
      ws->plans.erase(ws->plans.begin() + x--);
    }
    for (auto& pl : ws->plans) {
      if (pl->key != key) continue;
      pl->last_use = ws->uses;
      HIP_TRY(hipGraphLaunch(pl->pre, stream));
      HIP_TRY(hipEventRecord(ws->ev0, stream));
      HIP_TRY(launch_solve(pl->e, pl->workers, pl->tile, stream));
      HIP_TRY(hipEventRecord(ws->ev1, stream));
      HIP_TRY(hipGraphLaunch(pl->post, stream));
      HIP_TRY(hipStreamSynchronize(stream));
      return complete(ws, n, probs, o, ctx, pl->host_inst, pl->J, pl->widths, pl->coarse_engine,
                      pl->want_resid, pl->e.istat, stream, t0, stats, info, lk, true);
    }
  }
  std::unique_ptr<Plan> np(use_graph ? new Plan() : nullptr);

  // cell side per instance: the caller's, else (exact method) the tuned
  // table, keyed by the wall density of masked problems
  std::vector<double> density(n, 0.0);
  if (!o.cell && method == EIK_EXACT) {
    std::vector<WallIn> win;
    std::vector<int> which;
    int64_t wmax = 0;
    for (int k = 0; k < n; ++k) {
      if (!probs[k].mask) continue;
      if (ctx.density) {
        density[k] = ctx.density[k];
        continue;
      }
      if (!o.device_ptrs) {
        density[k] = wall_density_host(probs[k]);
        continue;
      }
      win.push_back(WallIn{probs[k].mask, probs[k].nx, probs[k].ny});
      which.push_back(k);
      wmax = std::max<int64_t>(wmax, (int64_t)probs[k].nx * probs[k].ny);
    }
    if (!win.empty()) {
      const int m = (int)win.size();
      HIP_TRY(ws->wall_in.ensure(m * sizeof(WallIn)));
      HIP_TRY(ws->wall_cnt.ensure(2 * m * sizeof(unsigned long long)));
      HIP_TRY(hipMemcpyAsync(ws->wall_in.p, win.data(), m * sizeof(WallIn), hipMemcpyHostToDevice, stream));
      HIP_TRY(hipMemsetAsync(ws->wall_cnt.p, 0, 2 * m * sizeof(unsigned long long), stream));
      HIP_TRY(launch_wall_density(ws->wall_in.as<WallIn>(), m, wmax,
                                  ws->wall_cnt.as<unsigned long long>(), stream));
      std::vector<unsigned long long> cnt(2 * m);
      HIP_TRY(hipMemcpyAsync(cnt.data(), ws->wall_cnt.p, cnt.size() * 8, hipMemcpyDeviceToHost, stream));
      HIP_TRY(hipStreamSynchronize(stream));
      for (int x = 0; x < m; ++x)
        density[which[x]] = cnt[2 * x] ? (double)cnt[2 * x + 1] / (double)cnt[2 * x] : 0.0;
    }
  }

  // tiling and sizes per instance
  std::vector<Inst> inst(n);
  std::vector<Tiling> til(n);
  int64_t total_nodes = 0, max_nodes = 0, max_src = 0;
  int extent = 0;
  // A launch sizes every wave's LDS for its widest cell: a batch keeps its
  // cells within 32 nodes (several waves per compute unit) unless every
  // problem asks for 64.
  std::vector<int> cells(n);
  bool all64 = true;
  for (int k = 0; k < n; ++k) {
    const eik_problem& p = probs[k];
    cells[k] = o.cell ? o.cell
                      : method == EIK_EXACT ? tuned_cell(dt, n > 1, p.nx, p.ny, density[k])
                                            : default_cell(p.nx, p.ny, method);
    all64 = all64 && cells[k] > 32;
  }
  if (!o.cell && method == EIK_EXACT && n > 1 && !all64)
    for (int& c : cells) c = std::min(c, 32);
  for (int k = 0; k < n; ++k) {
    const eik_problem& p = probs[k];
    const int s = cells[k];
    if ((rc = make_tiling(p.nx, p.ny, s, method, &til[k]))) return rc;
    extent = std::max(extent, til[k].extent);
    total_nodes += (int64_t)p.nx * p.ny;
    max_nodes = std::max<int64_t>(max_nodes, (int64_t)p.nx * p.ny);
    max_src = std::max<int64_t>(max_src, p.nsrc);
  }

  // staging of host inputs
  if (!dev) {
    int64_t nmask = 0, nsrc = 0;
    for (int k = 0; k < n; ++k) {
      nmask += probs[k].mask ? (int64_t)probs[k].nx * probs[k].ny : 0;
      nsrc += probs[k].nsrc;
    }
    HIP_TRY(ws->F.ensure(total_nodes * es));
    HIP_TRY(ws->u.ensure(total_nodes * es));
    HIP_TRY(ws->mask.ensure(nmask));
    HIP_TRY(ws->src.ensure(nsrc * sizeof(int64_t)));
    HIP_TRY(ws->q.ensure(nsrc * sizeof(double)));
  }
  if (!ctx.delta) HIP_TRY(ws->fine.delta.ensure(total_nodes * es));
  int64_t off = 0, moff = 0, soff = 0;
  for (int k = 0; k < n; ++k) {
    const eik_problem& p = probs[k];
    const int64_t nn = (int64_t)p.nx * p.ny;
    Inst& I = inst[k];
    std::memset(&I, 0, sizeof I);
    I.h = p.h;
    I.nx = p.nx;
    I.ny = p.ny;
    I.s = til[k].s;
    I.kx = til[k].kx;
    I.ky = til[k].ky;
    I.balanced = til[k].balanced;
    I.nsrc = p.nsrc;
    I.delta = ctx.delta ? ctx.delta[k] : (void*)(ws->fine.delta.as<char>() + off * es);
    if (dev) {
      I.u = p.u_out;
      I.F = p.F;
      I.mask = p.mask;
      I.src = p.src;
      I.q = p.q;
    } else {
      I.u = ws->u.as<char>() + off * es;
      I.F = ws->F.as<char>() + off * es;
      HIP_TRY(hipMemcpyAsync((void*)I.F, p.F, nn * es, hipMemcpyHostToDevice, stream));
      if (p.mask) {
        I.mask = ws->mask.as<uint8_t>() + moff;
        HIP_TRY(hipMemcpyAsync((void*)I.mask, p.mask, nn, hipMemcpyHostToDevice, stream));
        moff += nn;
      }
      I.src = ws->src.as<int64_t>() + soff;
      HIP_TRY(hipMemcpyAsync((void*)I.src, p.src, p.nsrc * sizeof(int64_t), hipMemcpyHostToDevice, stream));
      if (p.q) {
        I.q = ws->q.as<double>() + soff;
        HIP_TRY(hipMemcpyAsync((void*)I.q, p.q, p.nsrc * sizeof(double), hipMemcpyHostToDevice, stream));
      }
      soff += p.nsrc;
    }
    off += nn;
  }

  // band widths: the given one, else the tuned multiple of each problem's
  // own cell crossing at unit speed (s h)
  BandSpec bs{o.band > 0.0 ? o.band : 0.0, o.band_cells};
  int window = o.band_window;
  if (!(o.band > 0.0) && !(o.band_cells > 0.0)) tuned_band(method, dt, n > 1, &bs.cells, &window);
  std::vector<double> widths;
  if (sched == EIK_SCHED_BANDS)
    for (int k = 0; k < n; ++k) widths.push_back(bs.width_of(inst[k]));
  const uint64_t timeout = (uint64_t)ws->wall_khz * (uint64_t)(o.timeout_ms ? o.timeout_ms : 10000);
  int64_t J = 0;
  for (int k = 0; k < n; ++k) J += (int64_t)inst[k].kx * inst[k].ky;
  const int tile = tile_for(extent);
  if (extent > tile) return fail(EIK_EINVAL, "internal: a cell of %d nodes exceeds the %d-node tile", extent, tile);
  // the heap schedule has exactly one worker (it alone keeps the heap)
  const int workers =
      heap ? 1
           : o.workers ? o.workers
                       : std::max(1, default_workers(ws, J, tile, dt, method, n) / std::max(1, ctx.share));
  Engine e;
  // FIFO rings: for batches, one per 32 waves (at most kFifoRings); a single
  // problem keeps one ring (its few waves serve the narrow front best from
  // one queue: eight rings made the 4097^2 solve 3% slower, and the FP32
  // batch 5% faster)
  const int rings = n > 1 ? std::max(1, std::min<int>((int)kFifoRings, workers / 32)) : 1;
  if ((rc = setup_engine(ws->fine, inst, dt, method, dag, heap, widths.empty() ? nullptr : &bs, window,
                         o.eager_publish, o.max_cell_visits, timeout, stream, &e,
                         np ? &np->inst : nullptr, rings)))
    return rc;
  e.idone = ctx.idone;

  if (g_trace) {
    HIP_TRY(ws->ready_at.ensure(J * 8));
    HIP_TRY(ws->trace.ensure((size_t)kTraceCap * 64));
    HIP_TRY(ws->trace_n.ensure(4));
    HIP_TRY(hipMemsetAsync(ws->trace_n.p, 0, 4, stream));
    HIP_TRY(hipMemsetAsync(ws->ready_at.p, 0, J * 8, stream));
    e.ready_at = ws->ready_at.as<unsigned long long>();
    e.trace = ws->trace.as<unsigned long long>();
    e.trace_n = ws->trace_n.as<unsigned int>();
    e.trace_cap = kTraceCap;
  }
  Engine ce;
  int cw = 1;  // workers of the coarse cell engine
  // coarse grid of cell centres with spacing h^c = s h (FMSM Part I): FMSM
  // orders its cells by Fast Marching on it, as the method prescribes; the
  // other methods use the order only as a schedule and take a parallel exact
  // solve: Jacobi iteration in one workgroup per problem for coarse grids of
  // up to 1024 cells (a single problem: up to kCoarseJacobiMax), else the
  // cell engine (coarse_engine).  The 65 x 65 coarse grid of the 4097^2
  // checkerboard: 0.34 ms in the cell engine, ~0.26 ms by Jacobi; batches
  // keep the cell engine above 1024 cells (served mazes, whose coarse paths
  // wind, were ~3% slower by Jacobi)
  bool have_coarse = false, coarse_engine = false;
  const bool fmm = method == EIK_FMSM;
  int64_t max_coarse = 0;
  for (int k = 0; k < n; ++k) max_coarse = std::max<int64_t>(max_coarse, (int64_t)inst[k].kx * inst[k].ky);
  const bool jacobi = !fmm && max_coarse <= (n == 1 ? kCoarseJacobiMax : 1024);
  int cext = 0, fmm_lds = 0;
  FmmSpill spill{};
  if (dag) {
    HIP_TRY(ws->cF.ensure(J * sizeof(double)));
    HIP_TRY(ws->cmask.ensure(J));
    HIP_TRY(ws->cq.ensure(J * sizeof(double)));
    HIP_TRY(ws->cu.ensure(J * sizeof(double)));
    if (fmm) {
      HIP_TRY(ws->crank.ensure(J * sizeof(int32_t)));
      const int lim = coarse_fmm_lds_cells();
      int64_t big = 0;  // coarse cells of the problems that do not fit in LDS
      for (int k = 0; k < n; ++k) {
        const int64_t jk = (int64_t)inst[k].kx * inst[k].ky;
        if (jk <= lim) fmm_lds = std::max<int>(fmm_lds, (int)jk);
        else big = J;
      }
      if (big) {
        HIP_TRY(ws->fmm_spill.ensure(J * (2 * sizeof(double) + 2 * sizeof(int32_t))));
        spill.delta = ws->fmm_spill.as<double>();
        spill.fval = spill.delta + J;
        spill.st = reinterpret_cast<int32_t*>(spill.fval + J);
        spill.fidx = spill.st + J;
      }
    } else if (!jacobi) {
      HIP_TRY(ws->coarse.delta.ensure(J * sizeof(double)));
    }
    DevBuf& coutbuf = np ? np->cout : ws->cout;
    HIP_TRY(coutbuf.ensure(n * sizeof(CoarseOut)));
    std::vector<CoarseOut> co(n);
    std::vector<Inst> cinst(n);
    for (int k = 0; k < n; ++k) {
      const int64_t c0 = inst[k].cell0;
      co[k].F = ws->cF.as<double>() + c0;
      co[k].mask = ws->cmask.as<uint8_t>() + c0;
      co[k].q = ws->cq.as<double>() + c0;
      co[k].u = ws->cu.as<double>() + c0;
      co[k].rank = fmm ? ws->crank.as<int32_t>() + c0 : nullptr;
      if (fmm || jacobi) continue;
      Inst& C = cinst[k];
      std::memset(&C, 0, sizeof C);
      C.u = co[k].u;
      C.F = co[k].F;
      C.mask = co[k].mask;
      C.qdense = co[k].q;
      C.delta = ws->coarse.delta.as<double>() + c0;
      C.h = (double)inst[k].s * inst[k].h;
      C.nx = inst[k].kx;
      C.ny = inst[k].ky;
      Tiling ct;
      make_tiling(C.nx, C.ny, kCoarseEngineCell, EIK_EXACT, &ct);
      C.s = ct.s;
      C.kx = ct.kx;
      C.ky = ct.ky;
      C.balanced = ct.balanced;
      cext = std::max(cext, ct.extent);
    }
    HIP_TRY(hipMemcpyAsync(coutbuf.p, co.data(), n * sizeof(CoarseOut), hipMemcpyHostToDevice, stream));
    if (!fmm && !jacobi) {
      int64_t jc = 0;
      for (int k = 0; k < n; ++k) jc += (int64_t)cinst[k].kx * cinst[k].ky;
      cw = std::max(1, default_workers(ws, jc, tile_for(cext), EIK_F64, EIK_EXACT, n) / std::max(1, ctx.share));
      const int crings = n > 1 ? std::max(1, std::min<int>((int)kFifoRings, cw / 32)) : 1;
      if ((rc = setup_engine(ws->coarse, cinst, EIK_F64, EIK_EXACT, 0, 0, nullptr, 0, 0, 0, timeout, stream,
                             &ce, np ? &np->cinst : nullptr, crings)))
        return rc;
    }
    have_coarse = true;
    coarse_engine = !fmm && !jacobi;
  }
  const CoarseOut* co_dev = have_coarse ? (np ? np->cout : ws->cout).as<CoarseOut>() : nullptr;


  // The launch sequence: preparation (a1), coarse solve and ordering (a5),
  // the solver kernel between two timing events, residual and statistics
  // copy (a6).  With graph replay the parts before and after the solver
  // kernel are captured (on a private stream) into two graphs.
  const char* failed_step = "";
  hipError_t er = hipSuccess;
  auto step = [&](const char* what, hipError_t r) {
    if (er == hipSuccess && r != hipSuccess) {
      er = r;
      failed_step = what;
    }
  };
  auto pre = [&](hipStream_t ls) {
    step("prepare", launch_prepare(e, max_nodes, ls));
    if (have_coarse) {
      step("coarse inputs", launch_coarse_inputs(e, co_dev, (int)max_src, ls));
      if (jacobi) {
        step("coarse solve", launch_coarse_jacobi(e, co_dev, (int)max_coarse, ls));
      } else if (coarse_engine) {
        step("coarse prepare", launch_prepare(ce, J, ls));
        step("coarse solve", launch_solve(ce, cw, tile_for(cext), ls));
      } else {
        step("coarse fast marching", launch_coarse_fmm(e, co_dev, fmm_lds, spill, ls));
      }
      step("order", launch_dag(e, co_dev, (int)J, ls));
    }
  };
  auto post = [&](hipStream_t ls) {
    if (want_resid) step("residual", launch_residual(e, max_nodes, ls));
    step("statistics copy", hipMemcpyAsync(ws->ctl_host, e.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, ls));
    if (coarse_engine)
      step("coarse statistics copy",
           hipMemcpyAsync(ws->ctl_host + 1, ce.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, ls));
  };
  auto capture = [&](auto&& body, hipGraphExec_t* exec) -> int {
    HIP_TRY(hipStreamBeginCapture(ws->capture, hipStreamCaptureModeThreadLocal));
    body(ws->capture);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(ws->capture, &graph);
    if (er != hipSuccess || ec != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(EIK_EDEVICE, "graph capture failed (%s): %s", er != hipSuccess ? failed_step : "end",
                  hipGetErrorString(er != hipSuccess ? er : ec));
    }
    const hipError_t ei = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return fail(EIK_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
    return EIK_OK;
  };
  if (np) {
    if (!ws->capture) HIP_TRY(hipStreamCreateWithFlags(&ws->capture, hipStreamNonBlocking));
    if ((rc = capture(pre, &np->pre)) || (rc = capture(post, &np->post))) {
      drop_plan(np.get());
      return rc;
    }
    HIP_TRY(hipGraphLaunch(np->pre, stream));
  } else {
    pre(stream);
  }
  if (ws->ev0) step("event 0", hipEventRecord(ws->ev0, stream));
  step("solve", launch_solve(e, workers, tile, stream));
  if (ws->ev1) step("event 1", hipEventRecord(ws->ev1, stream));
  if (np) HIP_TRY(hipGraphLaunch(np->post, stream));
  else post(stream);
  if (er != hipSuccess) return fail(EIK_EDEVICE, "launch failed (%s): %s", failed_step, hipGetErrorString(er));
  if (np) {
    np->e = e;
    np->workers = workers;
    np->tile = tile;
    np->key = key;
    np->gen = ws->gen;
    np->last_use = ws->uses;
    np->host_inst = inst;
    np->J = J;
    np->widths = widths;
    np->coarse_engine = coarse_engine;
    np->want_resid = want_resid;
    if (ws->plans.size() >= kMaxPlans) {
      auto lru = std::min_element(ws->plans.begin(), ws->plans.end(),
                                  [](const std::unique_ptr<Plan>& a, const std::unique_ptr<Plan>& b) {
                                    return a->last_use < b->last_use;
                                  });
      drop_plan(lru->get());
      ws->plans.erase(lru);
    }
    ws->plans.push_back(std::move(np));
  }
  if (ctx.poll) {  // early completion: let the caller take finished problems
    for (;;) {
      const hipError_t q = hipStreamQuery(stream);
      if (q == hipSuccess) break;
      if (q != hipErrorNotReady) return fail(EIK_EDEVICE, "solve failed: %s", hipGetErrorString(q));
      ctx.poll(e, inst);
      std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    ctx.poll(e, inst);
  }
  HIP_TRY(hipStreamSynchronize(stream));
  return complete(ws, n, probs, o, ctx, inst, J, widths, coarse_engine, want_resid, e.istat, stream,
                  t0, stats, info, lk, false);
}

// After the solve's stream has completed: errors, FP32 certification (per
// problem), copies to host outputs, diagnostics and statistics.
static int complete(Workspace* ws, int n, const eik_problem* probs, const eik_opts& o,
                    const RunCtx& ctx, const std::vector<Inst>& inst, int64_t J, const std::vector<double>& widths,
                    bool coarse_engine, bool want_resid, const unsigned long long* istat,
                    hipStream_t stream, double t0, eik_stats* stats, RunInfo* info,
                    std::unique_lock<std::mutex>& lk, bool replayed) {
  const int dt = o.dtype;
  const size_t es = dsize(dt);
  const bool dev = o.device_ptrs != 0;
  int rc = EIK_OK;
  const Ctl c = ws->ctl_host[0];
  const unsigned err = c.err | (coarse_engine ? ws->ctl_host[1].err : 0u);
  if (err & (kErrSpeed | kErrSource))
    return fail(EIK_EINVAL, "%s", (err & kErrSpeed) ? "a speed value is not positive and finite"
                                                   : "a source is out of range, on an obstacle or has non-finite q");
  if (err & kErrGuard)
    return fail(EIK_ENOTCONV, "cell-visit guard tripped after %llu visits", (unsigned long long)c.visits);
  if (err & kErrDeadline) return fail(EIK_EDEVICE, "solver exceeded its time limit");
  float ms = 0.f;
  if (ws->ev0) HIP_TRY(hipEventElapsedTime(&ms, ws->ev0, ws->ev1));
  // per-problem counters and residuals (batches count per problem on the
  // device; a single problem's are the launch totals)
  std::vector<unsigned long long> is;
  if (n > 1 || want_resid) {
    is.resize(4 * (size_t)n);
    HIP_TRY(hipMemcpyAsync(is.data(), istat, is.size() * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
  }
  std::vector<double> resid(n, -1.0), resid32(n, -1.0);
  std::vector<int> fell(n, 0);
  if (want_resid)
    for (int k = 0; k < n; ++k) std::memcpy(&resid[k], &is[4 * (size_t)k + 3], sizeof(double));

  // FP32: certify each problem by its FP64 residual, else re-solve it in FP64
  if (dt == EIK_F32 && want_resid) {
    const double tol = o.residual_tol > 0.0 ? o.residual_tol : 4.0 * std::ldexp(1.0, -24);
    std::vector<int> which;
    for (int k = 0; k < n; ++k) {
      resid32[k] = resid[k];
      if (!(resid[k] <= tol) && !(ctx.detached && ctx.detached[k])) which.push_back(k);
    }
    if (!which.empty()) {
      std::vector<double> r64;
      lk.unlock();  // the FP64 solve takes the workspace lock itself
      rc = refine_fp64(which, probs, inst, o, stream, ctx, &r64);
      lk.lock();
      if (rc) return rc;
      for (size_t x = 0; x < which.size(); ++x) {
        fell[which[x]] = 1;
        resid[which[x]] = r64[x];
      }
    }
  }
  if (!dev) {
    for (int k = 0; k < n; ++k)
      HIP_TRY(hipMemcpyAsync(probs[k].u_out, inst[k].u, (size_t)probs[k].nx * probs[k].ny * es,
                             hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
  }
  if (g_profile) {
    const double us = 1e3 / ws->wall_khz;  // microseconds per tick
    std::fprintf(stderr,
                 "[eik profile] kernel %.1f us; wave-us idle %.0f claim %.0f load %.0f sweep %.0f "
                 "publish %.0f finish %.0f; visits %llu sweeps %llu checks %llu\n",
                 ms * 1e3, c.t_idle * us, c.t_claim * us, c.t_load * us, c.t_sweep * us,
                 c.t_publish * us, c.t_finish * us, (unsigned long long)c.visits,
                 (unsigned long long)c.sweeps, (unsigned long long)c.checks);
  }
  if (g_trace) {
    unsigned cnt = 0;
    HIP_TRY(hipMemcpy(&cnt, ws->trace_n.p, 4, hipMemcpyDeviceToHost));
    cnt = std::min(cnt, kTraceCap);
    std::vector<unsigned long long> t((size_t)cnt * 8);
    HIP_TRY(hipMemcpy(t.data(), ws->trace.p, t.size() * 8, hipMemcpyDeviceToHost));
    if (FILE* f = std::fopen(g_trace, "w")) {
      for (unsigned k = 0; k < cnt; ++k) {
        const unsigned long long* r = &t[(size_t)k * 8];
        std::fprintf(f, "%llu %llu %llu %llu %llu %llu %llu %llu %llu %llu\n", r[0] & 0xffffffffull,
                     (r[0] >> 32) & 0xffff, r[0] >> 48, r[1], r[2], r[3], r[4], r[5], r[6], r[7]);
      }
      std::fclose(f);
    }
  }
  if (info) {
    info->kernel_ms = ms;
    info->cells = J;
  }
  if (stats) {
    for (int k = 0; k < n; ++k) {
      eik_stats& S = stats[k];
      std::memset(&S, 0, sizeof S);
      S.seconds = now_s() - t0;
      S.kernel_seconds = ms * 1e-3;
      S.cells = (uint64_t)inst[k].kx * inst[k].ky;
      S.cell_visits = n > 1 ? is[4 * (size_t)k] : c.visits;
      S.sweeps = n > 1 ? is[4 * (size_t)k + 1] : c.sweeps;
      S.checks = n > 1 ? is[4 * (size_t)k + 2] : c.checks;
      S.band_steps = c.band_steps;
      S.mon_checks = c.mon_checks;
      S.mon_ok = c.mon_ok;
      S.max_residual = resid[k];
      S.cell_used = inst[k].s;
      S.band_used = widths.empty() ? -1.0 : widths[k];
      S.fell_back_to_f64 = fell[k];
      S.cells_total = (uint64_t)J;
      S.graph_replayed = replayed ? 1 : 0;
      S.residual_f32 = resid32[k];
    }
  }
  return EIK_OK;
}

// Re-solves FP32 problems in FP64 (speeds widened on the device) and rounds
// the results into their FP32 outputs (inst[k].u: device memory).  The FP64
// solve computes its own residual, which is returned per problem.
int refine_fp64(const std::vector<int>& which, const eik_problem* probs,
                const std::vector<Inst>& inst, const eik_opts& o, hipStream_t stream,
                const RunCtx& ctx, std::vector<double>* resid) {
  Workspace* ws = ctx.ws;
  const int m = (int)which.size();
  int64_t total = 0;
  for (int k : which) total += (int64_t)probs[k].nx * probs[k].ny;
  if (!ctx.f64) {
    std::lock_guard<std::mutex> lk(ws->mu);
    HIP_TRY(ws->F64.ensure(total * sizeof(double)));
    HIP_TRY(ws->u64.ensure(total * sizeof(double)));
  }
  std::vector<eik_problem> p64(m);
  std::vector<double*> u64(m);
  std::vector<void*> d64(m);
  int64_t off = 0;
  for (int x = 0; x < m; ++x) {
    const int k = which[x];
    const int64_t nn = (int64_t)probs[k].nx * probs[k].ny;
    double* F;
    if (ctx.f64) {
      F = static_cast<double*>(ctx.f64[k]);
      u64[x] = F + nn;
      d64[x] = F + 2 * nn;
    } else {
      F = ws->F64.as<double>() + off;
      u64[x] = ws->u64.as<double>() + off;
    }
    HIP_TRY(launch_convert(inst[k].F, EIK_F32, F, EIK_F64, nn, stream));
    p64[x] = probs[k];
    p64[x].F = F;
    p64[x].u_out = u64[x];
    p64[x].mask = inst[k].mask;
    p64[x].src = inst[k].src;
    p64[x].q = inst[k].q;
    off += nn;
  }
  eik_opts o64 = o;
  o64.dtype = EIK_F64;
  o64.device_ptrs = 1;
  o64.residual_check = 1;  // FP64: reported, never re-solved
  o64.graph = 0;
  RunCtx c64;
  c64.ws = ws;
  c64.delta = ctx.f64 ? d64.data() : nullptr;
  c64.share = ctx.share;
  std::vector<eik_stats> st(m);
  int rc = run(m, p64.data(), o64, st.data(), nullptr, &c64);
  if (rc) return rc;
  resid->resize(m);
  for (int x = 0; x < m; ++x) {
    const int k = which[x];
    const int64_t nn = (int64_t)probs[k].nx * probs[k].ny;
    HIP_TRY(launch_convert(u64[x], EIK_F64, inst[k].u, EIK_F32, nn, stream));
    (*resid)[x] = st[x].max_residual;
  }
  HIP_TRY(hipStreamSynchronize(stream));
  return EIK_OK;
}

}  // namespace eik

using namespace eik;

extern "C" {

int eik_solve(int32_t nx, int32_t ny, double h, const void* F, const uint8_t* mask, int32_t nsrc,
              const int64_t* src, const double* q, void* u_out, const eik_opts* opts,
              eik_stats* stats) {
  g_err.clear();
  eik_opts o = opts ? *opts : default_opts();
  int rc = check_opts(o);
  if (rc) return rc;
  eik_problem p{nx, ny, h, F, mask, nsrc, src, q, u_out};
  if ((rc = validate_shape(p))) return rc;
  if (!o.device_ptrs && (rc = validate_host(p, o.dtype))) return rc;
  if (o.device_ptrs && (rc = validate_device(p, o.dtype))) return rc;
  return run(1, &p, o, stats, nullptr);
}

int eik_solve_batched(int32_t n, const eik_problem* probs, const eik_opts* opts, eik_stats* stats) {
  g_err.clear();
  if (n < 1 || !probs) return fail(EIK_EINVAL, "empty batch");
  eik_opts o = opts ? *opts : default_opts();
  int rc = check_opts(o);
  if (rc) return rc;
  for (int k = 0; k < n; ++k) {
    if ((rc = validate_shape(probs[k]))) return fail(rc, "problem %d: %s", k, g_err.c_str());
    if (!o.device_ptrs && (rc = validate_host(probs[k], o.dtype)))
      return fail(rc, "problem %d: %s", k, g_err.c_str());
    if (o.device_ptrs && (rc = validate_device(probs[k], o.dtype)))
      return fail(rc, "problem %d: %s", k, g_err.c_str());
  }
  return run(n, probs, o, stats, nullptr);
}

int eik_probe_step_latency(int32_t dtype, int32_t side, int32_t sweeps, double* seconds) {
  g_err.clear();
  if ((dtype != EIK_F64 && dtype != EIK_F32) || (side != 32 && side != 64) || sweeps < 1 || !seconds)
    return fail(EIK_EINVAL, "dtype F64/F32, side 32 or 64, sweeps >= 1 and an output are required");
  Workspace* ws = nullptr;
  int rc = workspace(&ws);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(ws->mu);
  HIP_TRY(ws->sweep_stat.ensure(64));
  unsigned long long* t = ws->sweep_stat.as<unsigned long long>();
  HIP_TRY(launch_probe_sweep(dtype, side, 1, t, nullptr));  // warm-up
  HIP_TRY(launch_probe_sweep(dtype, side, sweeps, t, nullptr));
  unsigned long long ticks = 0;
  HIP_TRY(hipMemcpy(&ticks, t, sizeof ticks, hipMemcpyDeviceToHost));
  ticks &= ~(1ull << 63);
  *seconds = (double)ticks / ((double)ws->wall_khz * 1e3) / ((double)sweeps * (2 * side - 1));
  return EIK_OK;
}

const char* eik_last_error(void) { return g_err.c_str(); }

}  // extern "C"
