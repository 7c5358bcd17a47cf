// Device side of the 3-D exact solver (engine3.hip): arguments and launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eik {

constexpr int kCell3 = 8;  // nodes per cell edge
constexpr unsigned kErr3Speed = 1u, kErr3Source = 2u, kErr3Guard = 4u;

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
  int32_t* mark;         // per cell: the last round it was queued for
  int32_t* list_cur;     // cells of this round
  int32_t* list_next;    // cells queued for the next round ...
  int32_t* count_next;   // ... and their number
  unsigned* err;         // kErr3* bits
  unsigned long long* stats;  // [0] cell visits, [1] sweeps
};

// validation, h/F, u = +inf, exit nodes; queues round 1 (mark, list_next,
// count_next must start at zero)
hipError_t launch3_prepare(const Grid3& g, hipStream_t stream);
// processes the `cells` cells of g.list_cur as round `round`
hipError_t launch3_round(const Grid3& g, int cells, int round, hipStream_t stream);

}  // namespace eik
