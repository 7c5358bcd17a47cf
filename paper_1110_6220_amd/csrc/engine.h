// Internal interface between the C-ABI layer (api.cpp) and the HIP engine
// (engine.hip).  Not installed; the public interface is include/eik.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eik {

// Per-cell state word: bit 0 = queued (pending), bit 1 = being processed;
// bits 8..11 = preferred sweep directions raised by neighbours (0 SW, 1 NW,
// 2 NE, 3 SE).
constexpr uint32_t kPending = 1u;
constexpr uint32_t kRunning = 2u;
constexpr int kFlagShift = 8;
constexpr uint32_t kFlagMask = 0xFu << kFlagShift;

enum Method : int32_t { kExact = 0, kFmsm = 1, kFhcm = 2 };

// One problem instance.  Cell k along an axis of n nodes with K cells covers
// [lo(k), lo(k+1)) where lo(k) = k*s (and lo(K) = n) for the standard tiling,
// or floor(k*n/K) for the balanced one.
struct Inst {
  void* u;               // solution / working values (dtype)
  const void* F;         // speed (dtype)
  const uint8_t* mask;   // 1 accessible, 0 obstacle; nullptr = all accessible
  void* delta;           // workspace: h/F; +inf on obstacles and sources (dtype)
  const int64_t* src;    // exit-set nodes
  const double* q;       // exit costs, nullptr = 0
  double h;
  int32_t nx, ny;
  int32_t s;             // nominal cell side
  int32_t kx, ky;        // cells per axis
  int32_t balanced;      // tiling kind
  int32_t cell0;         // global id of the instance's first cell
  int32_t nsrc;
  int32_t pad;
};

// Multi-producer multi-consumer bucketed cell queue.  Bucket b holds a ring of
// `cap` slots; a slot is (sequence << 32 | cell).  Keys map to absolute band
// index floor(key / width); the ring is that index modulo nb.  `cursor` is the
// lowest absolute band that may hold work.
struct Queue {
  unsigned long long* slot;    // nb * cap
  unsigned long long* head;    // nb entries, stride kCtrStride
  unsigned long long* tail;    // nb entries, stride kCtrStride
  unsigned long long* cursor;  // 1
  uint32_t cap;                // power of two > number of cells
  uint32_t nb;                 // power of two
  double inv_width;            // 1 / band width (0: single band)
};
constexpr int kCtrStride = 16;  // 128 bytes between hot counters

// Device control block.
struct Ctl {
  unsigned long long active;      // cells pending or running
  unsigned long long visits;      // cell removals
  unsigned long long sweeps;      // productive sweeps
  unsigned long long checks;      // no-change sweeps
  unsigned long long band_steps;  // cursor advances
  unsigned long long mon_checks;
  unsigned long long mon_ok;
  unsigned long long resid_bits;  // max residual (bits of a non-negative double)
  unsigned long long guard;       // limit on total visits
  unsigned long long deadline;    // wall_clock64() value after which workers stop
  unsigned int err;               // bit 0 bad speed, 1 bad source, 2 guard, 3 deadline
  unsigned int done_waves;
  unsigned long long pad[4];
};
constexpr unsigned kErrSpeed = 1u, kErrSource = 2u, kErrGuard = 4u, kErrDeadline = 8u;

// Arguments of the engine kernels.
struct Engine {
  Inst* inst;            // device array (batched) -- may be null when ninst == 1
  Inst one;              // the instance when ninst == 1
  int32_t ninst;
  int32_t ncells;        // total cells J
  int32_t method;
  int32_t dtype;         // 0 f64, 1 f32
  uint32_t* st;          // J state words
  uint32_t* visits;      // J removal counts
  int32_t* cell_inst;    // J instance ids (batched only)
  unsigned int* key;     // J orderable bits of the float cell value
  Queue q;
  Ctl* ctl;
  unsigned long long guard;          // limit on total cell visits
  unsigned long long timeout_ticks;  // wall_clock64 ticks before workers give up
};

// Host-side launchers (engine.hip).  All work is enqueued on `stream`.
hipError_t launch_prepare(const Engine& e, int64_t total_nodes, hipStream_t stream);
hipError_t launch_solve(const Engine& e, int workers, int tile, hipStream_t stream);
hipError_t launch_residual(const Engine& e, int64_t total_nodes, hipStream_t stream);
size_t solve_lds_bytes(int dtype, int tile);

}  // namespace eik
