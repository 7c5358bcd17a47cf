// Three-dimensional exact solver of libeik for gfx950 (MI355X).
//
// The label-correcting method on cells (Algorithm generic_LC_cells; the
// Heap-Cell Method's exact variant), extended to a 3-D grid with six
// neighbours as the paper's conclusion proposes for its cell methods.  The
// Theorem of Section 3.2.1 -- any order of cell removals reaches the
// solution of the discrete system -- carries over unchanged, so the cells
// are processed in rounds: every cell queued for a round is processed at
// once (one wave per cell of 8 x 8 x 8 nodes), and a cell is queued for the
// next round when a node on a shared face decreased and is below the node
// across (the add criterion).  Rounds repeat until none is queued.
//
// In a cell, a Gauss-Seidel sweep in one of the eight orderings walks the
// anti-diagonal planes i + j + k = d of the tile: lane (ii, jj) owns a
// column and updates node kk = d - ii - jj, whose six neighbours lie on the
// planes d - 1 (upwind, written by the previous step) and d + 1 (old
// values).  A wave performs its LDS accesses in order, so the previous
// step's writes are visible without waiting; the order is a topological
// order of the lexicographic sweep, which it therefore equals.  Sweeps cycle
// through the orderings until one changes nothing.
#include <math.h>
#include <stdint.h>

#include "engine3.h"

namespace eik {
namespace {

constexpr int C3 = kCell3;   // nodes per cell edge
constexpr int P3 = C3 + 2;   // tile edge with the one-node halo

template <typename T>
__device__ __forceinline__ T ld_coh(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_coh(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The upwind update from the three axis minima, in the expression order of
// the CPU oracle (contraction disabled; sqrt correctly rounded): sorted
// m1 <= m2 <= m3; one-sided when m2 - m1 >= delta; else the two-sided root
// when it does not exceed m3; else the three-sided root of
// (U-m1)^2 + (U-m2)^2 + (U-m3)^2 = delta^2.
__device__ double update3(double a, double b, double c, double delta) {
  const double INF = __builtin_huge_val();
  const double lo = a < b ? a : b, hi = a < b ? b : a;
  const double m1 = lo < c ? lo : c, mid = lo < c ? c : lo;
  const double m2 = hi < mid ? hi : mid, m3 = hi < mid ? mid : hi;
  if (m1 == INF) return INF;
  const double d = m1 - m2;
  if (fabs(d) >= delta) return m1 + delta;
  const double u2 = 0.5 * (m1 + m2 + sqrt(2.0 * delta * delta - d * d));
  if (u2 <= m3) return u2;
  const double d13 = m1 - m3, d23 = m2 - m3;
  const double disc = 3.0 * delta * delta - (d * d + d13 * d13 + d23 * d23);
  if (!(disc >= 0.0)) return u2;
  return (m1 + m2 + m3 + sqrt(disc)) / 3.0;
}

__device__ __forceinline__ int cell_lo3(int c, int n) { return c * C3 < n ? c * C3 : n; }

// h/F on accessible nodes (validating F), +inf on obstacles; u = +inf.
__global__ void k3_prep(Grid3 g) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  bool bad = false;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x) {
    const bool acc = !g.mask || g.mask[x];
    double d = __builtin_huge_val();
    if (acc) {
      const double f = g.F[x];
      if (!(f > 0.0) || !isfinite(f)) bad = true;
      d = g.h / f;
    }
    g.delta[x] = d;
    g.u[x] = __builtin_huge_val();
  }
  if (bad) __hip_atomic_fetch_or(g.err, kErr3Speed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void atomic_min_d(double* p, double v) {
  unsigned long long* a = reinterpret_cast<unsigned long long*>(p);
  unsigned long long old = ld_coh(a);
  while (__builtin_bit_cast(double, old) > v) {
    if (__hip_atomic_compare_exchange_strong(a, &old, __builtin_bit_cast(unsigned long long, v),
                                             __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      break;
  }
}

// Queues cell c for round r (once per round).
__device__ __forceinline__ void queue3(const Grid3& g, int c, int r) {
  if (__hip_atomic_fetch_max(&g.mark[c], r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < r) {
    const int slot = __hip_atomic_fetch_add(g.count_next, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    g.list_next[slot] = c;
  }
}

// Exit nodes: validation, u = min q, frozen (delta = +inf); their cells and
// the six neighbouring cells are queued for round 1.
__global__ void k3_sources(Grid3 g) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < g.nsrc; s += gridDim.x * blockDim.x) {
    const int64_t x = g.src[s];
    const double q = g.q ? g.q[s] : 0.0;
    if (x < 0 || x >= n || (g.mask && !g.mask[x]) || !isfinite(q)) {
      __hip_atomic_fetch_or(g.err, kErr3Source, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      continue;
    }
    atomic_min_d(g.u + x, q);
    g.delta[x] = __builtin_huge_val();
    const int i = (int)(x % g.nx), j = (int)((x / g.nx) % g.ny), k = (int)(x / ((int64_t)g.nx * g.ny));
    const int cx = i / C3, cy = j / C3, cz = k / C3;
    const int c = (cz * g.ky + cy) * g.kx + cx;
    queue3(g, c, 1);
    if (cx > 0) queue3(g, c - 1, 1);
    if (cx + 1 < g.kx) queue3(g, c + 1, 1);
    if (cy > 0) queue3(g, c - g.kx, 1);
    if (cy + 1 < g.ky) queue3(g, c + g.kx, 1);
    if (cz > 0) queue3(g, c - g.kx * g.ky, 1);
    if (cz + 1 < g.kz) queue3(g, c + g.kx * g.ky, 1);
  }
}

// One round: the cells of list_cur, one wave each.
__global__ __launch_bounds__(64) void k3_round(Grid3 g, int round) {
  __shared__ double tu[P3 * P3 * P3];
  __shared__ double td[P3 * P3 * P3];
  __shared__ double u0[C3 * C3 * C3];
  const int lane = threadIdx.x;
  const double INF = __builtin_huge_val();
  const int c = g.list_cur[blockIdx.x];
  const int cx = c % g.kx, cy = (c / g.kx) % g.ky, cz = c / (g.kx * g.ky);
  const int x0 = cx * C3, y0 = cy * C3, z0 = cz * C3;
  const int w = cell_lo3(cx + 1, g.nx) - x0, hg = cell_lo3(cy + 1, g.ny) - y0,
            dp = cell_lo3(cz + 1, g.nz) - z0;
  const int64_t sxy = (int64_t)g.nx * g.ny;
  // the tile with its halo (the whole (C3+2)^3 block around the cell; edge
  // and corner halo values are loaded but never read)
  for (int t = lane; t < P3 * P3 * P3; t += 64) {
    const int a = t % P3 - 1, b = (t / P3) % P3 - 1, e = t / (P3 * P3) - 1;
    const int i = x0 + a, j = y0 + b, k = z0 + e;
    const bool in = a <= w && b <= hg && e <= dp && i >= 0 && j >= 0 && k >= 0 && i < g.nx &&
                    j < g.ny && k < g.nz;
    double v = INF, d = INF;
    if (in) {
      const int64_t x = k * sxy + (int64_t)j * g.nx + i;
      v = ld_coh(g.u + x);
      d = g.delta[x];
    }
    tu[t] = v;
    td[t] = d;
  }
  __syncthreads();
  for (int t = lane; t < C3 * C3 * C3; t += 64) {
    const int a = t % C3, b = (t / C3) % C3, e = t / (C3 * C3);
    u0[t] = tu[((e + 1) * P3 + b + 1) * P3 + a + 1];
  }
  __syncthreads();
  // sweeps until one changes nothing
  const int ii = lane % C3, jj = lane / C3;
  int nsw = 0;
  for (int sw = 0;; ++sw) {
    const int dir = sw & 7;
    const int sx = (dir & 1) ? -1 : 1, sy = (dir & 2) ? -1 : 1, sz = (dir & 4) ? -1 : 1;
    const int i = sx > 0 ? ii : w - 1 - ii, j = sy > 0 ? jj : hg - 1 - jj;
    const bool col = ii < w && jj < hg;
    bool changed = false;
    for (int d = 0; d < w + hg + dp - 2; ++d) {
      const int kk = d - ii - jj;
      if (col && kk >= 0 && kk < dp) {
        const int k = sz > 0 ? kk : dp - 1 - kk;
        const int t = ((k + 1) * P3 + j + 1) * P3 + i + 1;
        const double uW = tu[t - 1], uE = tu[t + 1], uS = tu[t - P3], uN = tu[t + P3];
        const double uD = tu[t - P3 * P3], uU = tu[t + P3 * P3];
        const double a = uW < uE ? uW : uE, b = uS < uN ? uS : uN, cc = uD < uU ? uD : uU;
        const double U = update3(a, b, cc, td[t]);
        if (U < tu[t]) {
          tu[t] = U;
          changed = true;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    ++nsw;
    if (__ballot(changed) == 0ull) break;
    if (sw > 4096) {  // a cell solve terminates; guard anyway
      __hip_atomic_fetch_or(g.err, kErr3Guard, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
  }
  __syncthreads();
  // write back the nodes that decreased
  for (int t = lane; t < C3 * C3 * C3; t += 64) {
    const int a = t % C3, b = (t / C3) % C3, e = t / (C3 * C3);
    if (a >= w || b >= hg || e >= dp) continue;
    const double v = tu[((e + 1) * P3 + b + 1) * P3 + a + 1];
    if (v < u0[t]) st_coh(g.u + (z0 + e) * sxy + (int64_t)(y0 + b) * g.nx + x0 + a, v);
  }
  __builtin_amdgcn_s_waitcnt(0);  // the stores complete before neighbours are queued
  __syncthreads();
  // add criterion per face: a face node that decreased and is below the node
  // across (accessible, not an exit node) queues the neighbouring cell
  for (int f = 0; f < 6; ++f) {
    const int ax = f >> 1, side = f & 1;
    const int n0 = ax == 0 ? hg : w, n1 = ax == 2 ? hg : dp;  // face extents
    const int lim = ax == 0 ? w : ax == 1 ? hg : dp;
    const int pos = side ? lim - 1 : 0, across = side ? lim : -1;
    bool q = false;
    for (int t = lane; t < n0 * n1; t += 64) {
      const int p0 = t % n0, p1 = t / n0;
      int a, b, e, aa, bb, ee;
      if (ax == 0) { a = pos; b = p0; e = p1; aa = across; bb = b; ee = e; }
      else if (ax == 1) { a = p0; b = pos; e = p1; aa = a; bb = across; ee = e; }
      else { a = p0; b = p1; e = pos; aa = a; bb = b; ee = across; }
      const double v = tu[((e + 1) * P3 + b + 1) * P3 + a + 1];
      const int ta = ((ee + 1) * P3 + bb + 1) * P3 + aa + 1;
      q = q || (v < u0[(e * C3 + b) * C3 + a] && td[ta] != INF && v < tu[ta]);
    }
    if (__ballot(q) != 0ull && lane == 0) {
      int nb = -1;
      if (ax == 0) nb = side ? (cx + 1 < g.kx ? c + 1 : -1) : (cx > 0 ? c - 1 : -1);
      if (ax == 1) nb = side ? (cy + 1 < g.ky ? c + g.kx : -1) : (cy > 0 ? c - g.kx : -1);
      if (ax == 2) nb = side ? (cz + 1 < g.kz ? c + g.kx * g.ky : -1) : (cz > 0 ? c - g.kx * g.ky : -1);
      if (nb >= 0) queue3(g, nb, round + 1);
    }
  }
  if (lane == 0) {
    __hip_atomic_fetch_add(&g.stats[0], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&g.stats[1], (unsigned long long)nsw, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  }
}

int grid_for3(int64_t n, int block, int cap) {
  int64_t b = (n + block - 1) / block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

}  // namespace

hipError_t launch3_prepare(const Grid3& g, hipStream_t stream) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL(k3_prep, dim3(grid_for3(n, 256, 8192)), dim3(256), 0, stream, g);
  hipLaunchKernelGGL(k3_sources, dim3(grid_for3(g.nsrc, 256, 1024)), dim3(256), 0, stream, g);
  return hipGetLastError();
}

hipError_t launch3_round(const Grid3& g, int cells, int round, hipStream_t stream) {
  hipLaunchKernelGGL(k3_round, dim3(cells), dim3(64), 0, stream, g, round);
  return hipGetLastError();
}

}  // namespace eik
