// Device side of the 3-D exact solver (engine3.hip): arguments and launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eik {

constexpr int kCell3 = 8;  // nodes per cell edge
constexpr unsigned kErr3Speed = 1u, kErr3Source = 2u, kErr3Guard = 4u, kErr3Count = 8u;

// One problem on an nx x ny x nz grid (node (i, j, k) at (k*ny + j)*nx + i),
// cut into kx x ky x kz cells of kCell3^3 nodes (the last ones ragged).
struct Grid3 {
  double* u;             // solution (device)
  const double* F;       // speed
  const uint8_t* mask;   // 1 accessible; nullptr = all accessible
  double* delta;         // workspace: h/F, +inf on obstacles and exit nodes
  const int64_t* src;    // exit nodes ...
  const double* q;       // ... and their costs (nullptr = 0)
  double h;
  int32_t nx, ny, nz, nsrc;
  int32_t kx, ky, kz;
  int32_t* mark;         // per cell: the last round it was queued for ...
  int32_t* entry;        // ... and the faces new values entered through
  int32_t* lists[2];     // round r processes lists[r & 1], queues into lists[(r + 1) & 1]
  int32_t* counts;       // [3]: round r's list length is counts[r % 3]
  int32_t* busy;         // rounds that processed at least one cell
  unsigned* err;         // kErr3* bits
  unsigned long long* stats;  // [0] cell visits, [1] sweeps
};

// validation, h/F, u = +inf, exit nodes; queues round 1 (mark, entry,
// lists, counts, busy must start at zero)
hipError_t launch3_prepare(const Grid3& g, hipStream_t stream);
// round `round` (>= 1): its list length is read on the device, so rounds can
// be enqueued without waiting; an empty round does nothing.  Each round also
// zeroes the counter the round after it queues into.  `blocks` waves loop
// over the list.  cap > 0: at most cap sweeps per visit; a cell not yet
// converged is listed again for the next round.
hipError_t launch3_round(const Grid3& g, int round, int blocks, int cap, hipStream_t stream);
// resident 64-thread blocks of the round kernel per compute unit
int round3_blocks_per_cu();

// ---- FMSM in three dimensions (cells as in Grid3) --------------------------
constexpr int kFront3 = 12288;  // coarse Fast Marching front held in LDS
constexpr unsigned kErr3Front = 16u;

struct Fmsm3 {
  double* Uc;        // coarse values
  double* dc;        // coarse h^c / F^c (+inf on coarse obstacles)
  double* cq;        // coarse exit cost: min q of the cell's exit nodes (+inf: none)
  uint8_t* lab;      // 0 far, 1 considered, 2 accepted
  uint8_t* cacc;     // the cell holds an accessible node
  int32_t* rank;     // processing position (-1: never processed)
  int32_t* level;    // level of the processing order's dependency graph (-1: never)
  int32_t* posf;     // position in the front
  int32_t* srcs;     // coarse exit cells, unordered ...
  int32_t* sorted;   // ... and by (cq, index)
  int32_t* ctl;      // [0] coarse exit cells, [1] levels, [2] processed cells
  unsigned long long* stats;  // [0] cells processed, [1] sweeps
  double hc;         // coarse spacing 8 h
};

// fine preparation (h/F, u = +inf, exit nodes), the coarse problem, the
// order of the coarse exit cells, and Fast Marching on the coarse grid (one
// wave): cell ranks and levels; f.ctl[1] = number of levels.  g.err and the
// f.ctl words must start at zero.
hipError_t launch3f_prepare(const Grid3& g, const Fmsm3& f, hipStream_t stream);
// Part II for the cells of one level (pairwise non-adjacent): `blocks` waves
hipError_t launch3f_level(const Grid3& g, const Fmsm3& f, int level, int blocks, hipStream_t stream);
int fmsm3_blocks_per_cu();

}  // namespace eik
