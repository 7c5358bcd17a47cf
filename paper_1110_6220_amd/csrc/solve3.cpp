// eik_solve3: the 3-D exact solver's host side -- validation, staging,
// preparation and the rounds of cell processing (engine3.hip).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "engine3.h"
#include "internal.h"

namespace eik {
namespace {

int validate3_host(int64_t n, const double* F, const uint8_t* mask, int32_t nsrc, const int64_t* src,
                   const double* q) {
  for (int64_t x = 0; x < n; ++x) {
    if (mask && !mask[x]) continue;
    if (!(F[x] > 0.0) || !std::isfinite(F[x]))
      return fail(EIK_EINVAL, "speed F[%lld] = %g is not positive and finite", (long long)x, F[x]);
  }
  for (int s = 0; s < nsrc; ++s) {
    if (src[s] < 0 || src[s] >= n) return fail(EIK_EINVAL, "source %d index %lld out of range", s, (long long)src[s]);
    if (mask && !mask[src[s]]) return fail(EIK_EINVAL, "source %d lies on an obstacle", s);
    if (q && !std::isfinite(q[s])) return fail(EIK_EINVAL, "source %d has non-finite q", s);
  }
  return EIK_OK;
}

// Fills the grid description and stages host inputs (device_ptrs = 0).
int stage3(Workspace* ws, int32_t nx, int32_t ny, int32_t nz, double h, const double* F,
           const uint8_t* mask, int32_t nsrc, const int64_t* src, const double* q, double* u_out,
           bool dev, hipStream_t stream, Grid3& g) {
  const int64_t n = (int64_t)nx * ny * nz;
  std::memset(&g, 0, sizeof g);
  g.h = h;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.nsrc = nsrc;
  g.kx = (nx + kCell3 - 1) / kCell3;
  g.ky = (ny + kCell3 - 1) / kCell3;
  g.kz = (nz + kCell3 - 1) / kCell3;
  if ((int64_t)g.kx * g.ky * g.kz > (1ll << 30)) return fail(EIK_EINVAL, "too many cells");
  if (dev) {
    g.u = u_out;
    g.F = F;
    g.mask = mask;
    g.src = src;
    g.q = q;
  } else {
    HIP_TRY(ws->F.ensure(n * sizeof(double)));
    HIP_TRY(ws->u.ensure(n * sizeof(double)));
    HIP_TRY(ws->src.ensure(nsrc * sizeof(int64_t)));
    HIP_TRY(hipMemcpyAsync(ws->F.p, F, n * sizeof(double), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(ws->src.p, src, nsrc * sizeof(int64_t), hipMemcpyHostToDevice, stream));
    g.u = ws->u.as<double>();
    g.F = ws->F.as<double>();
    g.src = ws->src.as<int64_t>();
    if (mask) {
      HIP_TRY(ws->mask.ensure(n));
      HIP_TRY(hipMemcpyAsync(ws->mask.p, mask, n, hipMemcpyHostToDevice, stream));
      g.mask = ws->mask.as<uint8_t>();
    }
    if (q) {
      HIP_TRY(ws->q.ensure(nsrc * sizeof(double)));
      HIP_TRY(hipMemcpyAsync(ws->q.p, q, nsrc * sizeof(double), hipMemcpyHostToDevice, stream));
      g.q = ws->q.as<double>();
    }
  }
  HIP_TRY(ws->fine.delta.ensure(n * sizeof(double)));
  g.delta = ws->fine.delta.as<double>();
  return EIK_OK;
}

int solve3(int32_t nx, int32_t ny, int32_t nz, double h, const double* F, const uint8_t* mask,
           int32_t nsrc, const int64_t* src, const double* q, double* u_out, bool dev,
           hipStream_t stream, eik3_stats* stats) {
  Workspace* ws = nullptr;
  int rc = workspace(&ws);
  if (rc) return rc;
  std::unique_lock<std::mutex> lk(ws->mu);
  const int64_t n = (int64_t)nx * ny * nz;
  Grid3 g;
  if ((rc = stage3(ws, nx, ny, nz, h, F, mask, nsrc, src, q, u_out, dev, stream, g))) return rc;
  const int64_t J = (int64_t)g.kx * g.ky * g.kz;
  // statistics (two 64-bit words, first so that their atomics are 8-byte
  // aligned: the allocation is 256-byte aligned), the three round counters,
  // the error word and the busy-round count; then per cell the mark, the
  // entry faces and the two lists
  constexpr size_t kHead = 64;
  HIP_TRY(ws->grid3.ensure(kHead + (size_t)J * 4 * sizeof(int32_t)));
  char* base = static_cast<char*>(ws->grid3.p);
  if (reinterpret_cast<uintptr_t>(base) % 8) return fail(EIK_EDEVICE, "workspace is not 8-byte aligned");
  g.stats = reinterpret_cast<unsigned long long*>(base);
  g.counts = reinterpret_cast<int32_t*>(base + 16);
  g.err = reinterpret_cast<unsigned*>(base + 28);
  g.busy = reinterpret_cast<int32_t*>(base + 32);
  g.mark = reinterpret_cast<int32_t*>(base + kHead);
  g.entry = g.mark + J;
  g.lists[0] = g.mark + 2 * J;
  g.lists[1] = g.mark + 3 * J;
  HIP_TRY(hipMemsetAsync(base, 0, kHead + (size_t)J * 4 * sizeof(int32_t), stream));
  const double t0 = now_s();
  HIP_TRY(launch3_prepare(g, stream));
  int32_t* hb = ws->host3;  // pinned: [0] a round's list length, [1] error word, [2] busy rounds
  HIP_TRY(hipMemcpyAsync(hb, &g.counts[1], sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(hb + 1, g.err, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  unsigned err = (unsigned)hb[1];
  if (err & (kErr3Speed | kErr3Source))
    return fail(EIK_EINVAL, "%s", (err & kErr3Speed) ? "a speed value is not positive and finite"
                                                    : "a source is out of range, on an obstacle or has non-finite q");
  // rounds are enqueued in batches; only the length of the list after a
  // batch comes back to the host (rounds past the last one are empty)
  const int64_t max_rounds = 16 * J + 64;
  const int blocks = (int)std::min<int64_t>(J, (int64_t)ws->cus * round3_blocks_per_cu());
  constexpr int kBatch = 8;
  // at most three sweeps per visit: a round lasts as long as its slowest
  // cell, and a cell still changing after three continues in the next round
  // (129^3: 4.4 -> 2.2 ms, 257^3: 11.7 -> 8.2 ms; two and four sweeps are slower)
  constexpr int kSweepCap = 3;
  int rounds = 0;
  int32_t pending = hb[0];
  HIP_TRY(hipEventRecord(ws->ev0, stream));
  while (pending > 0) {
    if (rounds > max_rounds) return fail(EIK_ENOTCONV, "round guard tripped after %d rounds", rounds);
    for (int b = 0; b < kBatch; ++b) HIP_TRY(launch3_round(g, ++rounds, blocks, kSweepCap, stream));
    HIP_TRY(hipMemcpyAsync(hb, &g.counts[(rounds + 1) % 3], sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(hb + 1, g.err, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if ((unsigned)hb[1] & kErr3Count) return fail(EIK_EDEVICE, "a round listed more than %lld cells", (long long)J);
    pending = hb[0];
  }
  HIP_TRY(hipEventRecord(ws->ev1, stream));
  unsigned long long st[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(&err, g.err, sizeof err, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(st, g.stats, sizeof st, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipMemcpyAsync(hb + 2, g.busy, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
  if (!dev) HIP_TRY(hipMemcpyAsync(u_out, g.u, n * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (err & kErr3Guard) return fail(EIK_ENOTCONV, "a cell's sweeps did not terminate");
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, ws->ev0, ws->ev1));
  if (stats) {
    stats->seconds = now_s() - t0;
    stats->rounds_seconds = ms * 1e-3;
    stats->rounds = hb[2];
    stats->cells = J;
    stats->cell_visits = (int64_t)st[0];
    stats->sweeps = (int64_t)st[1];
  }
  return EIK_OK;
}

// FMSM in three dimensions: preparation and coarse Fast Marching, then one
// launch per level of the processing order.
int fmsm3(int32_t nx, int32_t ny, int32_t nz, double h, const double* F, const uint8_t* mask,
          int32_t nsrc, const int64_t* src, const double* q, double* u_out, bool dev,
          hipStream_t stream, eik3_stats* stats) {
  Workspace* ws = nullptr;
  int rc = workspace(&ws);
  if (rc) return rc;
  std::unique_lock<std::mutex> lk(ws->mu);
  const int64_t n = (int64_t)nx * ny * nz;
  Grid3 g;
  if ((rc = stage3(ws, nx, ny, nz, h, F, mask, nsrc, src, q, u_out, dev, stream, g))) return rc;
  const int64_t J = (int64_t)g.kx * g.ky * g.kz;
  // head (statistics first: 8-byte aligned, the allocation is 256-byte
  // aligned; counters; error word), then per cell Uc, dc, cq (doubles), rank,
  // level, posf, srcs, sorted (int32), lab, cacc (bytes)
  constexpr size_t kHead = 64;
  const size_t bytes = kHead + (size_t)J * (3 * sizeof(double) + 5 * sizeof(int32_t) + 2);
  HIP_TRY(ws->fmsm3.ensure(bytes));
  char* base = static_cast<char*>(ws->fmsm3.p);
  if (reinterpret_cast<uintptr_t>(base) % 8) return fail(EIK_EDEVICE, "workspace is not 8-byte aligned");
  Fmsm3 f;
  f.stats = reinterpret_cast<unsigned long long*>(base);
  f.ctl = reinterpret_cast<int32_t*>(base + 16);
  g.err = reinterpret_cast<unsigned*>(base + 28);
  double* d = reinterpret_cast<double*>(base + kHead);
  f.Uc = d;
  f.dc = d + J;
  f.cq = d + 2 * J;
  int32_t* w = reinterpret_cast<int32_t*>(d + 3 * J);
  f.rank = w;
  f.level = w + J;
  f.posf = w + 2 * J;
  f.srcs = w + 3 * J;
  f.sorted = w + 4 * J;
  f.lab = reinterpret_cast<uint8_t*>(w + 5 * J);
  f.cacc = f.lab + J;
  f.hc = (double)kCell3 * h;
  HIP_TRY(hipMemsetAsync(base, 0, kHead, stream));
  const double t0 = now_s();
  HIP_TRY(hipEventRecord(ws->ev0, stream));
  HIP_TRY(launch3f_prepare(g, f, stream));
  int32_t* hb = ws->host3;  // pinned: the 32-byte head
  HIP_TRY(hipMemcpyAsync(hb, base, 32, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  unsigned err = (unsigned)hb[7];
  if (err & (kErr3Speed | kErr3Source))
    return fail(EIK_EINVAL, "%s", (err & kErr3Speed) ? "a speed value is not positive and finite"
                                                    : "a source is out of range, on an obstacle or has non-finite q");
  if (err & kErr3Front)
    return fail(EIK_ENOMEM, "the coarse Fast Marching front outgrew its %d entries", kFront3);
  const int levels = hb[5];
  const int blocks = (int)std::min<int64_t>(J, (int64_t)ws->cus * fmsm3_blocks_per_cu());
  for (int L = 0; L < levels; ++L) HIP_TRY(launch3f_level(g, f, L, blocks, stream));
  HIP_TRY(hipEventRecord(ws->ev1, stream));
  HIP_TRY(hipMemcpyAsync(hb, base, 32, hipMemcpyDeviceToHost, stream));
  if (!dev) HIP_TRY(hipMemcpyAsync(u_out, g.u, n * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if ((unsigned)hb[7] & kErr3Guard) return fail(EIK_ENOTCONV, "a cell's sweeps did not terminate");
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, ws->ev0, ws->ev1));
  if (stats) {
    const unsigned long long* st = reinterpret_cast<const unsigned long long*>(hb);
    stats->seconds = now_s() - t0;
    stats->rounds_seconds = ms * 1e-3;
    stats->rounds = levels;
    stats->cells = J;
    stats->cell_visits = (int64_t)st[0];
    stats->sweeps = (int64_t)st[1];
  }
  return EIK_OK;
}

}  // namespace
}  // namespace eik

using namespace eik;

static int check3(int32_t nx, int32_t ny, int32_t nz, double h, const double* F, const uint8_t* mask,
                  int32_t nsrc, const int64_t* src, const double* q, double* u_out, int32_t device_ptrs) {
  g_err.clear();
  if (nx < 1 || ny < 1 || nz < 1) return fail(EIK_EINVAL, "grid %d x %d x %d is empty", nx, ny, nz);
  if ((long long)nx * ny * nz > (1ll << 31) - 1) return fail(EIK_EINVAL, "grid too large");
  if (!(h > 0.0) || !std::isfinite(h)) return fail(EIK_EINVAL, "h = %g must be positive and finite", h);
  if (!F || !u_out) return fail(EIK_EINVAL, "F and u_out are required");
  if (nsrc < 1 || !src) return fail(EIK_EINVAL, "at least one source is required");
  if (device_ptrs != 0 && device_ptrs != 1) return fail(EIK_EINVAL, "device_ptrs must be 0 or 1");
  if (device_ptrs) {
    const auto off = [](const void* p, size_t a) { return reinterpret_cast<uintptr_t>(p) % a != 0; };
    if (off(F, 8) || off(u_out, 8) || off(src, 8) || (q && off(q, 8)))
      return fail(EIK_EINVAL, "F, u_out, src and q must be 8-byte aligned");
    return EIK_OK;
  }
  return validate3_host((int64_t)nx * ny * nz, F, mask, nsrc, src, q);
}

extern "C" int eik_solve3(int32_t nx, int32_t ny, int32_t nz, double h, const double* F,
                          const uint8_t* mask, int32_t nsrc, const int64_t* src, const double* q,
                          double* u_out, int32_t device_ptrs, void* stream, eik3_stats* stats) {
  const int rc = check3(nx, ny, nz, h, F, mask, nsrc, src, q, u_out, device_ptrs);
  if (rc) return rc;
  return solve3(nx, ny, nz, h, F, mask, nsrc, src, q, u_out, device_ptrs != 0,
                static_cast<hipStream_t>(stream), stats);
}

extern "C" int eik_fmsm3(int32_t nx, int32_t ny, int32_t nz, double h, const double* F,
                         const uint8_t* mask, int32_t nsrc, const int64_t* src, const double* q,
                         double* u_out, int32_t device_ptrs, void* stream, eik3_stats* stats) {
  const int rc = check3(nx, ny, nz, h, F, mask, nsrc, src, q, u_out, device_ptrs);
  if (rc) return rc;
  return fmsm3(nx, ny, nz, h, F, mask, nsrc, src, q, u_out, device_ptrs != 0,
               static_cast<hipStream_t>(stream), stats);
}
