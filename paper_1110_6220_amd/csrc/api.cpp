// C-ABI layer of libeik: argument validation, per-device workspace, staging of
// host buffers, launch sequencing and statistics.  Declarations and the
// contract of every entry point are in include/eik.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/eik.h"
#include "engine.h"

namespace {

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

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(EIK_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t need) {
    if (need <= bytes) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    size_t b = std::max<size_t>(need, 256);
    hipError_t e = hipMalloc(&p, b);
    if (e == hipSuccess) bytes = b;
    return e;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

// Workspace of one device: reused by every call on that device.
struct Workspace {
  std::mutex mu;
  DevBuf delta, st, visits, cell_inst, key, slot, head, tail, cursor, ctl, inst;
  // staging for host pointers
  DevBuf F, u, mask, src, q;
  eik::Ctl* ctl_host = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int cus = 0;
  int wall_khz = 0;
  bool ready = false;
};

std::mutex g_ws_mu;
std::vector<std::unique_ptr<Workspace>> g_ws;

int workspace(Workspace** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_ws_mu);
  if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
  if (!g_ws[dev]) g_ws[dev].reset(new Workspace());
  Workspace* w = g_ws[dev].get();
  if (!w->ready) {
    HIP_TRY(hipHostMalloc((void**)&w->ctl_host, sizeof(eik::Ctl), hipHostMallocDefault));
    HIP_TRY(hipEventCreate(&w->ev0));
    HIP_TRY(hipEventCreate(&w->ev1));
    HIP_TRY(hipDeviceGetAttribute(&w->cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipDeviceGetAttribute(&w->wall_khz, hipDeviceAttributeWallClockRate, dev));
    if (w->wall_khz <= 0) w->wall_khz = 100000;
    w->ready = true;
  }
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
  if (o.workers < 0) return fail(EIK_EINVAL, "workers must be >= 0");
  if (o.method != EIK_EXACT)
    return fail(EIK_EINVAL, "method %d is not available in this build", (int)o.method);
  return EIK_OK;
}

// Standard tiling: K = ceil(n/s) cells of s nodes, a last cell of one node
// merged into its predecessor.  If that leaves a cell wider than 64 nodes the
// exact method uses the balanced tiling (K = ceil(n/s) cells of floor/ceil
// n/K nodes); its result does not depend on the tiling.
struct Tiling {
  int s, kx, ky, balanced, extent;
};

int std_cells(int n, int s) {
  int K = (n + s - 1) / s;
  if (K > 1 && n % s == 1) K--;
  return K;
}

int make_tiling(int nx, int ny, int s, int method, Tiling* t) {
  t->s = s;
  t->kx = std_cells(nx, s);
  t->ky = std_cells(ny, s);
  int ex = std::max({std::min(s, nx), nx - (t->kx - 1) * s, std::min(s, ny), ny - (t->ky - 1) * s});
  t->balanced = 0;
  if (ex > 64) {
    if (method != EIK_EXACT)
      return fail(EIK_EINVAL, "cell side %d leaves a cell of %d nodes (> 64) for this method", s, ex);
    t->kx = (nx + s - 1) / s;
    t->ky = (ny + s - 1) / s;
    t->balanced = 1;
    ex = std::max((nx + t->kx - 1) / t->kx, (ny + t->ky - 1) / t->ky);
  }
  t->extent = ex;
  return EIK_OK;
}

int tile_for(int extent) { return extent <= 16 ? 16 : extent <= 32 ? 32 : 64; }

int default_cell(int nx, int ny) {
  const int n = std::max(nx, ny);
  return n >= 512 ? 64 : n >= 160 ? 32 : 16;
}

uint32_t pow2_at_least(uint64_t v) {
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

int validate_shape(const eik_problem& p) {
  if (p.nx < 1 || p.ny < 1) return fail(EIK_EINVAL, "grid %d x %d is empty", p.nx, p.ny);
  if ((long long)p.nx * p.ny > (1ll << 31) - 1) return fail(EIK_EINVAL, "grid too large");
  if (!(p.h > 0.0) || !std::isfinite(p.h)) return fail(EIK_EINVAL, "h = %g must be positive and finite", p.h);
  if (!p.F || !p.u_out) return fail(EIK_EINVAL, "F and u_out are required");
  if (p.nsrc < 1 || !p.src) return fail(EIK_EINVAL, "at least one source is required");
  return EIK_OK;
}

// ---------------------------------------------------------------------------
// the solve driver shared by eik_solve and eik_solve_batched
// ---------------------------------------------------------------------------

int run(int n, const eik_problem* probs, const eik_opts& o, eik_stats* stats) {
  const double t0 = now_s();
  Workspace* ws = nullptr;
  int rc = workspace(&ws);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(ws->mu);
  hipStream_t stream = static_cast<hipStream_t>(o.stream);
  const int dt = o.dtype;
  const size_t es = dsize(dt);

  // tiling and sizes per instance
  std::vector<eik::Inst> inst(n);
  std::vector<Tiling> til(n);
  int64_t total_nodes = 0, max_nodes = 0, total_cells = 0, max_src = 0;
  int extent = 0;
  for (int k = 0; k < n; ++k) {
    const eik_problem& p = probs[k];
    const int s = o.cell ? o.cell : default_cell(p.nx, p.ny);
    if ((rc = make_tiling(p.nx, p.ny, s, o.method, &til[k]))) return rc;
    extent = std::max(extent, til[k].extent);
    total_nodes += (int64_t)p.nx * p.ny;
    max_nodes = std::max<int64_t>(max_nodes, (int64_t)p.nx * p.ny);
    total_cells += (int64_t)til[k].kx * til[k].ky;
    max_src = std::max<int64_t>(max_src, p.nsrc);
  }
  if (total_cells > (1ll << 30)) return fail(EIK_EINVAL, "too many cells");

  // staging of host inputs
  const bool dev = o.device_ptrs != 0;
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
  HIP_TRY(ws->delta.ensure(total_nodes * es));
  int64_t off = 0, moff = 0, soff = 0;
  int64_t cell0 = 0;
  for (int k = 0; k < n; ++k) {
    const eik_problem& p = probs[k];
    const int64_t nn = (int64_t)p.nx * p.ny;
    eik::Inst& I = inst[k];
    std::memset(&I, 0, sizeof I);
    I.h = p.h;
    I.nx = p.nx;
    I.ny = p.ny;
    I.s = til[k].s;
    I.kx = til[k].kx;
    I.ky = til[k].ky;
    I.balanced = til[k].balanced;
    I.cell0 = (int32_t)cell0;
    I.nsrc = p.nsrc;
    I.delta = ws->delta.as<char>() + off * es;
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
    cell0 += (int64_t)I.kx * I.ky;
  }

  // cell state, queue, control block
  const uint32_t J = (uint32_t)total_cells;
  double band = o.band;
  if (band == 0.0) {
    // default band: one cell crossing at unit speed
    double hs = 0.0;
    for (int k = 0; k < n; ++k) hs = std::max(hs, probs[k].h * til[k].s);
    band = hs;
  }
  const uint32_t nb = band > 0.0 ? 64u : 1u;
  const uint32_t cap = pow2_at_least((uint64_t)J + 1);
  HIP_TRY(ws->st.ensure(J * sizeof(uint32_t)));
  HIP_TRY(ws->visits.ensure(J * sizeof(uint32_t)));
  HIP_TRY(ws->key.ensure(J * sizeof(uint32_t)));
  HIP_TRY(ws->cell_inst.ensure(n > 1 ? J * sizeof(int32_t) : 4));
  HIP_TRY(ws->slot.ensure((size_t)cap * nb * sizeof(unsigned long long)));
  HIP_TRY(ws->head.ensure((size_t)nb * eik::kCtrStride * sizeof(unsigned long long)));
  HIP_TRY(ws->tail.ensure((size_t)nb * eik::kCtrStride * sizeof(unsigned long long)));
  HIP_TRY(ws->cursor.ensure(128));
  HIP_TRY(ws->ctl.ensure(sizeof(eik::Ctl)));
  if (n > 1) {
    HIP_TRY(ws->inst.ensure(n * sizeof(eik::Inst)));
    HIP_TRY(hipMemcpyAsync(ws->inst.p, inst.data(), n * sizeof(eik::Inst), hipMemcpyHostToDevice, stream));
  }

  eik::Engine e;
  std::memset(&e, 0, sizeof e);
  e.inst = n > 1 ? ws->inst.as<eik::Inst>() : nullptr;
  e.one = inst[0];
  e.ninst = n;
  e.ncells = (int32_t)J;
  e.method = o.method;
  e.dtype = dt;
  e.st = ws->st.as<uint32_t>();
  e.visits = ws->visits.as<uint32_t>();
  e.cell_inst = ws->cell_inst.as<int32_t>();
  e.key = ws->key.as<unsigned int>();
  e.q.slot = ws->slot.as<unsigned long long>();
  e.q.head = ws->head.as<unsigned long long>();
  e.q.tail = ws->tail.as<unsigned long long>();
  e.q.cursor = ws->cursor.as<unsigned long long>();
  e.q.cap = cap;
  e.q.nb = nb;
  e.q.inv_width = band > 0.0 ? 1.0 / band : 0.0;
  e.ctl = ws->ctl.as<eik::Ctl>();
  e.guard = o.max_cell_visits ? o.max_cell_visits : 64ull * J + 1024ull;
  e.timeout_ticks = (unsigned long long)ws->wall_khz * 1000ull * 10ull;  // 10 s

  const int tile = tile_for(extent);
  int workers = o.workers;
  if (workers == 0) {
    const int per_cu = tile == 64 ? (dt == EIK_F64 ? 2 : 4) : tile == 32 ? 8 : 16;
    workers = (int)std::min<int64_t>(J, (int64_t)ws->cus * per_cu);
    if (n == 1) workers = std::min(workers, 256);
  }
  workers = std::max(workers, 1);

  HIP_TRY(eik::launch_prepare(e, max_nodes, stream));
  HIP_TRY(hipEventRecord(ws->ev0, stream));
  HIP_TRY(eik::launch_solve(e, workers, tile, stream));
  HIP_TRY(hipEventRecord(ws->ev1, stream));
  const bool want_resid = o.residual_check != 0;
  if (want_resid) HIP_TRY(eik::launch_residual(e, max_nodes, stream));
  HIP_TRY(hipMemcpyAsync(ws->ctl_host, e.ctl, sizeof(eik::Ctl), hipMemcpyDeviceToHost, stream));
  if (!dev) {
    for (int k = 0; k < n; ++k)
      HIP_TRY(hipMemcpyAsync(probs[k].u_out, inst[k].u, (size_t)probs[k].nx * probs[k].ny * es,
                             hipMemcpyDeviceToHost, stream));
  }
  HIP_TRY(hipStreamSynchronize(stream));
  const eik::Ctl& c = *ws->ctl_host;
  if (c.err & (eik::kErrSpeed | eik::kErrSource))
    return fail(EIK_EINVAL, "%s", (c.err & eik::kErrSpeed) ? "a speed value is not positive and finite"
                                                          : "a source is out of range, on an obstacle or has non-finite q");
  if (c.err & eik::kErrGuard)
    return fail(EIK_ENOTCONV, "cell-visit guard tripped after %llu visits", (unsigned long long)c.visits);
  if (c.err & eik::kErrDeadline) return fail(EIK_EDEVICE, "solver exceeded its time limit");
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, ws->ev0, ws->ev1));
  if (stats) {
    for (int k = 0; k < (stats ? n : 0); ++k) {
      eik_stats& S = stats[k];
      std::memset(&S, 0, sizeof S);
      S.seconds = now_s() - t0;
      S.kernel_seconds = ms * 1e-3;
      S.cells = (uint64_t)inst[k].kx * inst[k].ky;
      S.cell_visits = c.visits;
      S.sweeps = c.sweeps;
      S.checks = c.checks;
      S.band_steps = c.band_steps;
      S.mon_checks = c.mon_checks;
      S.mon_ok = c.mon_ok;
      double r;
      std::memcpy(&r, &c.resid_bits, sizeof r);
      S.max_residual = want_resid ? r : -1.0;
      S.cell_used = inst[k].s;
      S.band_used = band;
      S.fell_back_to_f64 = 0;
    }
  }
  return EIK_OK;
}

}  // namespace

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
  return run(1, &p, o, stats);
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
  }
  return run(n, probs, o, stats);
}

const char* eik_last_error(void) { return g_err.c_str(); }

}  // extern "C"
