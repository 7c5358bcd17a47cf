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
// across (the add criterion).  Rounds repeat until none is queued.  Queueing
// a cell once per round coalesces the requests of all its neighbours: a
// queue served as soon as a request arrives (persistent waves) processes a
// cell before its other upwind faces have settled and visits each cell
// several times more.
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

// Lists cell c for round r (once per round: its mark).
__device__ __forceinline__ void enlist3(const Grid3& g, int c, int r) {
  if (__hip_atomic_fetch_max(&g.mark[c], r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < r) {
    const int slot = __hip_atomic_fetch_add(&g.counts[r % 3], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    g.lists[r & 1][slot] = c;
  }
}
// Queues cell c for round r, recording the face the new values enter
// through (bit 2 * axis + side, side 1 = the cell's high face): the cell's
// first sweep runs away from it.
__device__ __forceinline__ void queue3(const Grid3& g, int c, int r, int face) {
  __hip_atomic_fetch_or(&g.entry[c], 1 << face, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  enlist3(g, c, r);
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
    enlist3(g, c, 1);
    if (cx > 0) queue3(g, c - 1, 1, 1);
    if (cx + 1 < g.kx) queue3(g, c + 1, 1, 0);
    if (cy > 0) queue3(g, c - g.kx, 1, 3);
    if (cy + 1 < g.ky) queue3(g, c + g.kx, 1, 2);
    if (cz > 0) queue3(g, c - g.kx * g.ky, 1, 5);
    if (cz + 1 < g.kz) queue3(g, c + g.kx * g.ky, 1, 4);
  }
}

// One round: the cells of lists[round & 1], one wave each (a block takes
// every gridDim.x-th entry).  A visit loads the (C3+2)^3 block around the
// cell (u) and h/F of the cell into LDS, sweeps until a sweep changes
// nothing, stores the nodes that decreased and applies the add criterion on
// the six faces.
__global__ __launch_bounds__(64) void k3_round(Grid3 g, int round) {
  __shared__ double tu[P3 * P3 * P3];      // u on the cell and its one-node halo
  __shared__ double td[C3 * C3 * C3];      // h/F on the cell
  __shared__ uint8_t dec[C3 * C3 * C3];    // the node decreased in this visit
  const int lane = threadIdx.x;
  const double INF = __builtin_huge_val();
  const int64_t sxy = (int64_t)g.nx * g.ny;
  const int n = ld_coh(&g.counts[round % 3]);
  if (blockIdx.x == 0 && lane == 0) {
    st_coh(&g.counts[(round + 2) % 3], 0);  // round - 1's count: the queue of round + 1
    if (n > 0) __hip_atomic_fetch_add(g.busy, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (n > g.kx * g.ky * g.kz) {  // a cell is listed at most once per round
    if (blockIdx.x == 0 && lane == 0)
      __hip_atomic_fetch_or(g.err, kErr3Count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  unsigned long long nvis = 0, nsw = 0;  // this wave's totals
  for (int idx = blockIdx.x; idx < n; idx += gridDim.x) {
    const int c = g.lists[round & 1][idx];
    int entry = 0;
    if (lane == 0) entry = __hip_atomic_exchange(&g.entry[c], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    entry = __builtin_amdgcn_readfirstlane(entry);
    const int cx = c % g.kx, cy = (c / g.kx) % g.ky, cz = c / (g.kx * g.ky);
    const int x0 = cx * C3, y0 = cy * C3, z0 = cz * C3;
    const int w = cell_lo3(cx + 1, g.nx) - x0, hg = cell_lo3(cy + 1, g.ny) - y0,
              dp = cell_lo3(cz + 1, g.nz) - z0;
    // all loads of a lane in flight at once
    constexpr int NT = (P3 * P3 * P3 + 63) / 64, ND = C3 * C3 * C3 / 64;
    double vu[NT], vd[ND];
#pragma unroll
    for (int r = 0; r < NT; ++r) {
      const int t = lane + 64 * r;
      const int a = t % P3 - 1, b = (t / P3) % P3 - 1, e = t / (P3 * P3) - 1;
      const int i = x0 + a, j = y0 + b, k = z0 + e;
      const bool in = t < P3 * P3 * P3 && a <= w && b <= hg && e <= dp && i >= 0 && j >= 0 &&
                      k >= 0 && i < g.nx && j < g.ny && k < g.nz;
      vu[r] = in ? ld_coh(g.u + (k * sxy + (int64_t)j * g.nx + i)) : INF;
    }
#pragma unroll
    for (int r = 0; r < ND; ++r) {
      const int t = lane + 64 * r;
      const int a = t % C3, b = (t / C3) % C3, e = t / (C3 * C3);
      const bool in = a < w && b < hg && e < dp;
      vd[r] = in ? g.delta[(z0 + e) * sxy + (int64_t)(y0 + b) * g.nx + x0 + a] : INF;
    }
#pragma unroll
    for (int r = 0; r < NT; ++r)
      if (lane + 64 * r < P3 * P3 * P3) tu[lane + 64 * r] = vu[r];
#pragma unroll
    for (int r = 0; r < ND; ++r) {
      td[lane + 64 * r] = vd[r];
      dec[lane + 64 * r] = 0;
    }
    __syncthreads();
    // first ordering: along each axis away from the face the values entered
    // through (when exactly one of its two faces); axes without such a face
    // are the first to change direction in later sweeps
    int base = 0, ord[3], nf = 0;
    for (int ax = 0; ax < 3; ++ax) {
      const int lo = (entry >> (2 * ax)) & 1, hi = (entry >> (2 * ax + 1)) & 1;
      if (hi && !lo) base |= 1 << ax;
      if (lo == hi) ord[nf++] = ax;
    }
    for (int ax = 0, m = nf; ax < 3; ++ax) {
      const int lo = (entry >> (2 * ax)) & 1, hi = (entry >> (2 * ax + 1)) & 1;
      if (lo != hi) ord[m++] = ax;
    }
    // sweeps until one changes nothing
    const int ii = lane % C3, jj = lane / C3;
    for (int sw = 0;; ++sw) {
      const int dir = base ^ ((sw & 1) << ord[0]) ^ (((sw >> 1) & 1) << ord[1]) ^ (((sw >> 2) & 1) << ord[2]);
      const int sx = (dir & 1) ? -1 : 1, sy = (dir & 2) ? -1 : 1, sz = (dir & 4) ? -1 : 1;
      const int i = sx > 0 ? ii : w - 1 - ii, j = sy > 0 ? jj : hg - 1 - jj;
      const bool col = ii < w && jj < hg;
      bool changed = false;
      for (int d = 0; d < w + hg + dp - 2; ++d) {
        const int kk = d - ii - jj;
        if (col && kk >= 0 && kk < dp) {
          const int k = sz > 0 ? kk : dp - 1 - kk;
          const int t = ((k + 1) * P3 + j + 1) * P3 + i + 1, ci = (k * C3 + j) * C3 + i;
          const double uW = tu[t - 1], uE = tu[t + 1], uS = tu[t - P3], uN = tu[t + P3];
          double dl = td[ci];
          const double uD = tu[t - P3 * P3], uU = tu[t + P3 * P3], uo = tu[t];
          asm volatile("" : "+v"(dl));  // h/F joins the neighbours' LDS round trip
          const double a = uW < uE ? uW : uE, b = uS < uN ? uS : uN, cc = uD < uU ? uD : uU;
          const double U = update3(a, b, cc, dl);
          if (U < uo) {
            tu[t] = U;
            dec[ci] = 1;
            changed = true;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
      ++nsw;
      if (__ballot(changed) == 0ull) break;
      if (sw > 4096) {  // a cell solve terminates; guard anyway
        if (lane == 0) __hip_atomic_fetch_or(g.err, kErr3Guard, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    ++nvis;
    __syncthreads();
    // write back the nodes that decreased
#pragma unroll
    for (int r = 0; r < ND; ++r) {
      const int t = lane + 64 * r;
      const int a = t % C3, b = (t / C3) % C3, e = t / (C3 * C3);
      if (a < w && b < hg && e < dp && dec[t])
        st_coh(g.u + (z0 + e) * sxy + (int64_t)(y0 + b) * g.nx + x0 + a,
               tu[((e + 1) * P3 + b + 1) * P3 + a + 1]);
    }
    __builtin_amdgcn_s_waitcnt(0);  // the stores complete before neighbours are queued
    __syncthreads();
    // add criterion per face: a face node that decreased and is below the
    // node across (accessible, not an exit node: finite h/F) queues the
    // neighbour
    for (int f = 0; f < 6; ++f) {
      const int ax = f >> 1, side = f & 1;
      int nb = -1;
      if (ax == 0) nb = side ? (cx + 1 < g.kx ? c + 1 : -1) : (cx > 0 ? c - 1 : -1);
      if (ax == 1) nb = side ? (cy + 1 < g.ky ? c + g.kx : -1) : (cy > 0 ? c - g.kx : -1);
      if (ax == 2) nb = side ? (cz + 1 < g.kz ? c + g.kx * g.ky : -1) : (cz > 0 ? c - g.kx * g.ky : -1);
      if (nb < 0) continue;  // no cell across: the across plane is outside the grid
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
        if (!dec[(e * C3 + b) * C3 + a]) continue;
        const double v = tu[((e + 1) * P3 + b + 1) * P3 + a + 1];
        if (v < tu[((ee + 1) * P3 + bb + 1) * P3 + aa + 1] &&
            g.delta[(z0 + ee) * sxy + (int64_t)(y0 + bb) * g.nx + x0 + aa] != INF)
          q = true;
      }
      if (__ballot(q) != 0ull && lane == 0) queue3(g, nb, round + 1, 2 * ax + (1 - side));
    }
    __syncthreads();  // the next cell reuses the LDS arrays
  }
  if (lane == 0 && nvis) {
    __hip_atomic_fetch_add(&g.stats[0], nvis, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&g.stats[1], nsw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

hipError_t launch3_round(const Grid3& g, int round, int blocks, hipStream_t stream) {
  hipLaunchKernelGGL(k3_round, dim3(blocks), dim3(64), 0, stream, g, round);
  return hipGetLastError();
}

int round3_blocks_per_cu() {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void*>(k3_round), 64, 0) !=
          hipSuccess || b < 1)
    b = 1;
  return b;
}

}  // namespace eik
