// Whole-grid sweeping on the device: Fast Sweeping and Locking Sweeping (the
// prior methods of Section 2, Algorithm FSM) one sweep at a time, with the
// early termination studied in the Section 4 remark on stopping sweeping
// methods before convergence.  The preparation (h/F, exit nodes, validation)
// is the cell solver's; each sweep is one launch per tile anti-diagonal.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace eik {
namespace {

int check_sweep_opts(const eik_sweep_opts& o) {
  if (o.dtype != EIK_F64 && o.dtype != EIK_F32) return fail(EIK_EINVAL, "unknown dtype %d", (int)o.dtype);
  if (o.locking != 0 && o.locking != 1) return fail(EIK_EINVAL, "locking must be 0 or 1");
  if (o.max_sweeps < 0) return fail(EIK_EINVAL, "max_sweeps %d is negative", o.max_sweeps);
  if (std::isnan(o.threshold)) return fail(EIK_EINVAL, "threshold is NaN");
  return EIK_OK;
}

int sweep_solve(const eik_problem& p, const eik_sweep_opts& o, double* max_change,
                int64_t* n_changed, eik_sweep_stats* stats) {
  Workspace* ws = nullptr;
  int rc = workspace(&ws);
  if (rc) return rc;
  std::unique_lock<std::mutex> lk(ws->mu);
  hipStream_t stream = static_cast<hipStream_t>(o.stream);
  const int dt = o.dtype;
  const size_t es = dsize(dt);
  const bool dev = o.device_ptrs != 0;
  const int64_t nn = (int64_t)p.nx * p.ny;
  const int max_sweeps = o.max_sweeps ? o.max_sweeps : 65536;

  Inst I;
  std::memset(&I, 0, sizeof I);
  I.h = p.h;
  I.nx = p.nx;
  I.ny = p.ny;
  I.s = kSweepTile;
  I.kx = (p.nx + kSweepTile - 1) / kSweepTile;
  I.ky = (p.ny + kSweepTile - 1) / kSweepTile;
  I.balanced = 0;
  I.nsrc = p.nsrc;
  if (dev) {
    I.u = p.u_out;
    I.F = p.F;
    I.mask = p.mask;
    I.src = p.src;
    I.q = p.q;
  } else {
    HIP_TRY(ws->F.ensure(nn * es));
    HIP_TRY(ws->u.ensure(nn * es));
    HIP_TRY(ws->src.ensure(p.nsrc * sizeof(int64_t)));
    I.u = ws->u.p;
    I.F = ws->F.p;
    I.src = ws->src.as<int64_t>();
    HIP_TRY(hipMemcpyAsync(ws->F.p, p.F, nn * es, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(ws->src.p, p.src, p.nsrc * sizeof(int64_t), hipMemcpyHostToDevice, stream));
    if (p.mask) {
      HIP_TRY(ws->mask.ensure(nn));
      I.mask = ws->mask.as<uint8_t>();
      HIP_TRY(hipMemcpyAsync(ws->mask.p, p.mask, nn, hipMemcpyHostToDevice, stream));
    }
    if (p.q) {
      HIP_TRY(ws->q.ensure(p.nsrc * sizeof(double)));
      I.q = ws->q.as<double>();
      HIP_TRY(hipMemcpyAsync(ws->q.p, p.q, p.nsrc * sizeof(double), hipMemcpyHostToDevice, stream));
    }
  }
  HIP_TRY(ws->fine.delta.ensure(nn * es));
  I.delta = ws->fine.delta.p;
  std::vector<Inst> inst{I};
  Engine e;
  const uint64_t timeout = (uint64_t)ws->wall_khz * 10000ull;
  if ((rc = setup_engine(ws->fine, inst, dt, EIK_EXACT, 0, 0, nullptr, 0, 0, 0, timeout, stream, &e))) return rc;
  const int kx = I.kx, ky = I.ky, J = kx * ky;
  HIP_TRY(ws->sweep_stat.ensure(4 * sizeof(unsigned long long)));
  HIP_TRY(ws->sweep_dirty.ensure(J));
  HIP_TRY(launch_prepare(e, nn, stream));
  if (o.locking) {
    HIP_TRY(hipMemsetAsync(ws->sweep_dirty.p, 0, J, stream));
    HIP_TRY(launch_sweep_seed(e, p.nsrc, ws->sweep_dirty.as<uint8_t>(), stream));
  }
  // device-side validation of the inputs
  HIP_TRY(hipMemcpyAsync(ws->ctl_host, e.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (ws->ctl_host[0].err & (kErrSpeed | kErrSource))
    return fail(EIK_EINVAL, "%s", (ws->ctl_host[0].err & kErrSpeed)
                                      ? "a speed value is not positive and finite"
                                      : "a source is out of range, on an obstacle or has non-finite q");

  SweepArgs a;
  std::memset(&a, 0, sizeof a);
  a.stat = ws->sweep_stat.as<unsigned long long>();
  a.dirty = ws->sweep_dirty.as<uint8_t>();
  a.locking = o.locking;
  int done = 0, converged = 0;
  int64_t swept = 0, skipped = 0;
  float total_ms = 0.f;
  for (int k = 0; k < max_sweeps; ++k) {
    HIP_TRY(hipMemsetAsync(a.stat, 0, 4 * sizeof(unsigned long long), stream));
    HIP_TRY(hipEventRecord(ws->ev0, stream));
    a.dir = k & 3;
    for (int d = 0; d < kx + ky - 1; ++d) {
      a.diag = d;
      const int tiles = std::min(d, kx - 1) - std::max(0, d - (ky - 1)) + 1;
      HIP_TRY(launch_sweep_diag(e, a, tiles, stream));
    }
    HIP_TRY(hipEventRecord(ws->ev1, stream));
    unsigned long long st[4];
    HIP_TRY(hipMemcpyAsync(st, a.stat, sizeof st, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ws->ev0, ws->ev1));
    total_ms += ms;
    double mx;
    std::memcpy(&mx, &st[0], sizeof mx);
    if (max_change) max_change[k] = mx;
    if (n_changed) n_changed[k] = (int64_t)st[1];
    swept += (int64_t)st[2];
    skipped += (int64_t)st[3];
    ++done;
    if (st[1] == 0) {
      converged = 1;
      break;
    }
    if (o.threshold >= 0.0 && mx <= o.threshold) break;
  }
  if (!dev) {
    HIP_TRY(hipMemcpyAsync(p.u_out, I.u, nn * es, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
  }
  if (stats) {
    stats->sweeps = done;
    stats->converged = converged;
    stats->seconds = total_ms * 1e-3;
    stats->tiles_swept = swept;
    stats->tiles_skipped = skipped;
  }
  return EIK_OK;
}

}  // namespace
}  // namespace eik

using namespace eik;

extern "C" int eik_sweep_solve(int32_t nx, int32_t ny, double h, const void* F, const uint8_t* mask,
                               int32_t nsrc, const int64_t* src, const double* q, void* u_out,
                               const eik_sweep_opts* opts, double* max_change, int64_t* n_changed,
                               eik_sweep_stats* stats) {
  g_err.clear();
  eik_sweep_opts o;
  std::memset(&o, 0, sizeof o);
  if (opts) o = *opts;
  int rc = check_sweep_opts(o);
  if (rc) return rc;
  eik_problem p{nx, ny, h, F, mask, nsrc, src, q, u_out};
  if ((rc = validate_shape(p))) return rc;
  if (!o.device_ptrs && (rc = validate_host(p, o.dtype))) return rc;
  if (o.device_ptrs && (rc = validate_device(p, o.dtype))) return rc;
  return sweep_solve(p, o, max_change, n_changed, stats);
}
