// eik_solve_noalloc: eik_solve without any device allocation.
//
// Every device buffer the solver needs beyond the caller's inputs and
// outputs -- h/F per node, cell states, visit counts, cell values, the
// queue, counters, the coarse grid of the cell order -- is carved out of one
// file-scope device array, `scratch`, instead of the library's workspace
// (which grows with hipMalloc).  Each device that runs this entry point
// holds its own copy of the array for the life of the process; its address
// is taken once per device with hipGetSymbolAddress and only that address is
// used from the host.  Calls on one device share the array: they are
// serialised by the device's lock, and each call re-initialises everything
// it reads on the device (the preparation kernels), so the previous call's
// contents never leak into a result.
#include <hip/hip_runtime.h>

#include <cstring>
#include <memory>
#include <mutex>

#include "../../include/eik.h"
#include "internal.h"

namespace eik {
namespace {

constexpr size_t kScratchBytes = EIK_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct NoAlloc {
  std::once_flag once;
  int rc = EIK_OK;
  std::string err;
  void* ptr = nullptr;  // this device's copy of `scratch`
  Bump bump;
  Workspace ws;
  Ctl ctl_host[2];      // statistics read-back (pageable host memory)
};
NoAlloc g_na[kMaxDevices];

// Once per device, with the device current: the device address of its
// scratch array, and a workspace whose buffers are carved from it.
int na_init(int dev, NoAlloc** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(EIK_EDEVICE, "device %d out of range", dev);
  NoAlloc& na = g_na[dev];
  std::call_once(na.once, [&na] {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      na.rc = EIK_EDEVICE;
      na.err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
      return;
    }
    na.ptr = p;
    na.bump.base = static_cast<char*>(p);
    na.bump.cap = kScratchBytes;
    na.ws.bump = &na.bump;
    na.ws.ctl_host = na.ctl_host;
    const int rc = workspace_init(&na.ws);  // no allocation with a bump workspace
    if (rc) {
      na.rc = rc;
      na.err = g_err;
    }
  });
  if (na.rc) return fail(na.rc, "%s", na.err.c_str());
  *out = &na;
  return EIK_OK;
}

// Conservative device bytes of one solve: h/F per node plus the per-cell
// arrays, the queue rings and the coarse grid (256-byte alignment of every
// buffer included).
size_t scratch_need(int64_t nodes, int64_t J, int dtype, int nbands) {
  size_t cap = 1;
  while (cap < (size_t)J + 1) cap <<= 1;
  if (nbands == 1) {  // the FIFO's rings
    size_t rc = 1;
    while (rc < (size_t)(J + kFifoRings - 1) / kFifoRings + 1) rc <<= 1;
    cap = rc * kFifoRings;
  }
  // states, visits, values, dependency counts, order bits, heap blocks;
  // coarse speed, mask, exit cost, value, rank, h/F and Fast Marching spill
  const size_t per_cell = 4 + 4 + 8 + 4 + 1 + 1 + 8 + 1 + 8 + 8 + 4 + 8 + 24;
  return (size_t)nodes * (dtype == EIK_F64 ? 8 : 4) + (size_t)J * per_cell +
         (size_t)nbands * cap * 8 + (size_t)(nbands + kFifoRings) * 3 * 128 + 64 * 256 + (1u << 16);
}

}  // namespace
}  // namespace eik

using namespace eik;

extern "C" int eik_solve_noalloc(int32_t nx, int32_t ny, double h, const void* F,
                                 const uint8_t* mask, int32_t nsrc, const int64_t* src,
                                 const double* q, void* u_out, const eik_opts* opts,
                                 eik_stats* stats) {
  g_err.clear();
  eik_opts o = opts ? *opts : default_opts();
  int rc = check_opts(o);
  if (rc) return rc;
  if (!o.device_ptrs) return fail(EIK_EINVAL, "eik_solve_noalloc takes device pointers only");
  if (o.graph) return fail(EIK_EINVAL, "eik_solve_noalloc does not capture graphs");
  if (o.dtype == EIK_F32 && o.residual_check)
    return fail(EIK_EINVAL, "eik_solve_noalloc has no FP64 re-solve (residual_check with F32)");
  eik_problem p{nx, ny, h, F, mask, nsrc, src, q, u_out};
  if ((rc = validate_shape(p))) return rc;
  if ((rc = validate_device(p, o.dtype))) return rc;
  const int s = o.cell ? o.cell : 16;  // the smallest tuned side has the most cells
  Tiling t;
  if ((rc = make_tiling(nx, ny, s, o.method, &t))) return rc;
  const int64_t J = (int64_t)t.kx * t.ky;
  const int sched = o.schedule ? o.schedule : (o.method == EIK_FHCM ? EIK_SCHED_BANDS : EIK_SCHED_COARSE);
  const size_t need = scratch_need((int64_t)nx * ny, J, o.dtype, sched == EIK_SCHED_BANDS ? 64 : 1);
  if (need > kScratchBytes)
    return fail(EIK_EINVAL, "a %d x %d grid needs about %zu bytes of scratch; the allocation-free "
                "entry point holds %zu", nx, ny, need, kScratchBytes);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  NoAlloc* na = nullptr;
  if ((rc = na_init(dev, &na))) return rc;
  RunCtx ctx;
  ctx.ws = &na->ws;
  rc = run(1, &p, o, stats, nullptr, &ctx);
  if (rc && na->bump.overflow) {
    (void)hipStreamSynchronize(static_cast<hipStream_t>(o.stream));
    return fail(EIK_ENOMEM, "the problem exceeds the %zu-byte scratch of eik_solve_noalloc",
                kScratchBytes);
  }
  return rc;
}
