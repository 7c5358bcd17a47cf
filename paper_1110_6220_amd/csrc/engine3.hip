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
// through the orderings until one changes nothing, at most a capped number
// per visit: a cell still changing is listed again for the next round.
#include <math.h>
#include <stdint.h>

#include "engine3.h"
#include "wave.h"

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
// accesses to data that only one workgroup touches while the kernel runs:
// the compute unit's caches serve them
template <typename T>
__device__ __forceinline__ T ld_wg(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ void st_wg(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The upwind update from the three axis minima, in the expression order of
// the CPU oracle (contraction disabled; sqrt correctly rounded): sorted
// m1 <= m2 <= m3; one-sided when m2 - m1 >= delta; else the two-sided root
// when it does not exceed m3; else the three-sided root of
// (U-m1)^2 + (U-m2)^2 + (U-m3)^2 = delta^2.
__device__ double update3(double a, double b, double c, double delta) {
  const double INF = __builtin_huge_val();
  // sorting network on single min/max instructions (operands are never NaN)
  const double lo = wave::vmin(a, b), hi = wave::vmax(a, b);
  const double m1 = wave::vmin(lo, c), mid = wave::vmax(lo, c);
  const double m2 = wave::vmin(hi, mid), m3 = wave::vmax(hi, mid);
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
__global__ __launch_bounds__(64) void k3_round(Grid3 g, int round, int cap) {
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
    // sweeps until one changes nothing (at most `cap` per visit when cap > 0)
    const int ii = lane % C3, jj = lane / C3;
    bool again = false;
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
          const double a = wave::vmin(uW, uE), b = wave::vmin(uS, uN), cc = wave::vmin(uD, uU);
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
      if (sw + 1 == cap) {  // not yet converged: the cell continues in the next round
        again = true;
        break;
      }
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
    // neighbour; the six neighbours are queued by six lanes at once
    unsigned qmask = 0;
    for (int f = 0; f < 6; ++f) {
      const int ax = f >> 1, side = f & 1;
      const bool has = ax == 0 ? (side ? cx + 1 < g.kx : cx > 0)
                               : ax == 1 ? (side ? cy + 1 < g.ky : cy > 0) : (side ? cz + 1 < g.kz : cz > 0);
      if (!has) continue;  // no cell across: the across plane is outside the grid
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
      if (__ballot(q) != 0ull) qmask |= 1u << f;
    }
    if (lane < 6 && ((qmask >> lane) & 1u)) {
      const int ax = lane >> 1, side = lane & 1;
      const int nb = c + (side ? 1 : -1) * (ax == 0 ? 1 : ax == 1 ? g.kx : g.kx * g.ky);
      queue3(g, nb, round + 1, 2 * ax + (1 - side));
    }
    if (again && lane == 0) {  // the same entry faces, so that its next visit starts alike
      __hip_atomic_fetch_or(&g.entry[c], entry, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      enlist3(g, c, round + 1);
    }
    __syncthreads();  // the next cell reuses the LDS arrays
  }
  if (lane == 0 && nvis) {
    __hip_atomic_fetch_add(&g.stats[0], nvis, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&g.stats[1], nsw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// FMSM in three dimensions (Algorithm FMSM extended as Section 5 proposes)
// ---------------------------------------------------------------------------

// Canonical order of the eight orderings (bit 0 x descending, bit 1 y
// descending, bit 2 z descending): z ascending first, each z direction with
// the 2-D order SW, NW, NE, SE: 0, 2, 3, 1, 4, 6, 7, 5.
__device__ __forceinline__ int seq3(int q) { return (0x57641320u >> (4 * q)) & 7; }

// Orderings allowed for a cell whose earlier-processed neighbours lie on
// `faces` (bit 2 axis + side), in a grid one node thick along `thin` (bit
// axis): per axis the ascending direction for a low face, the descending
// one for a high face, both for both or none; ascending only on a thin axis.
__device__ __forceinline__ uint32_t orderings3(int faces, int thin) {
  int allow[3];
  for (int a = 0; a < 3; ++a) {
    const int lo = (faces >> (2 * a)) & 1, hi = (faces >> (2 * a + 1)) & 1;
    allow[a] = (thin >> a) & 1 ? 1 : (lo || hi) ? (lo ? 1 : 0) | (hi ? 2 : 0) : 3;
  }
  uint32_t m = 0;
  for (int d = 0; d < 8; ++d)
    if (((allow[0] >> (d & 1)) & (allow[1] >> ((d >> 1) & 1)) & (allow[2] >> ((d >> 2) & 1)) & 1) != 0)
      m |= 1u << d;
  return m;
}

// One Gauss-Seidel sweep of the cell in LDS in ordering dir, anti-diagonal
// planes (lane = (i, j) column); DIRECTIONAL: the update from the ordering's
// three upwind neighbours only.  Returns whether a node decreased (wave-wide).
template <bool DIRECTIONAL>
__device__ __forceinline__ bool sweep_cell3(double* tu, const double* td, uint8_t* dec, int dir, int w,
                                            int hg, int dp, int lane) {
  const int ii = lane % C3, jj = lane / C3;
  const int sx = (dir & 1) ? -1 : 1, sy = (dir & 2) ? -1 : 1, sz = (dir & 4) ? -1 : 1;
  const int i = sx > 0 ? ii : w - 1 - ii, j = sy > 0 ? jj : hg - 1 - jj;
  const bool col = ii < w && jj < hg;
  bool changed = false;
  for (int d = 0; d < w + hg + dp - 2; ++d) {
    const int kk = d - ii - jj;
    if (col && kk >= 0 && kk < dp) {
      const int k = sz > 0 ? kk : dp - 1 - kk;
      const int t = ((k + 1) * P3 + j + 1) * P3 + i + 1, ci = (k * C3 + j) * C3 + i;
      double dl = td[ci];
      double a, b, cc;
      const double uo = tu[t];
      if constexpr (DIRECTIONAL) {
        a = tu[t - sx];
        b = tu[t - sy * P3];
        cc = tu[t - sz * P3 * P3];
      } else {
        const double uW = tu[t - 1], uE = tu[t + 1], uS = tu[t - P3], uN = tu[t + P3];
        const double uD = tu[t - P3 * P3], uU = tu[t + P3 * P3];
        a = wave::vmin(uW, uE);
        b = wave::vmin(uS, uN);
        cc = wave::vmin(uD, uU);
      }
      asm volatile("" : "+v"(dl));  // h/F joins the neighbours' LDS round trip
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
  return __ballot(changed) != 0ull;
}

__device__ __forceinline__ int nb_cell3(const Grid3& g, int c, int e) {
  const int cx = c % g.kx, cy = (c / g.kx) % g.ky, cz = c / (g.kx * g.ky);
  switch (e) {
    case 0: return cx > 0 ? c - 1 : -1;
    case 1: return cx + 1 < g.kx ? c + 1 : -1;
    case 2: return cy > 0 ? c - g.kx : -1;
    case 3: return cy + 1 < g.ky ? c + g.kx : -1;
    case 4: return cz > 0 ? c - g.kx * g.ky : -1;
    default: return cz + 1 < g.kz ? c + g.kx * g.ky : -1;
  }
}

// wave-wide maximum of small integers (DPP row exchanges)
__device__ __forceinline__ int wave_max_i(int v) { return -wave::min_i(-v); }

__global__ void k3f_init(Grid3 g, Fmsm3 f) {
  const int J = g.kx * g.ky * g.kz;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < J; c += gridDim.x * blockDim.x)
    f.cq[c] = __builtin_huge_val();
}

// Exit nodes: validation, u = min q, frozen (h/F = +inf); the coarse exit
// cost of their cell (min q).
__global__ void k3f_sources(Grid3 g, Fmsm3 f) {
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
    atomic_min_d(f.cq + ((k / C3) * g.ky + j / C3) * g.kx + i / C3, q);
  }
}

// The coarse problem, one thread per cell: accessible or not; coarse speed F
// at the cell centre (the mean of the accessible ones among the one or two
// middle nodes per axis, added x outermost, then y, then z), else the mean of
// F over the cell (each x-plane y outer, z inner, then the planes x
// ascending); h^c / F^c; coarse exit cells listed.
__global__ void k3f_coarse(Grid3 g, Fmsm3 f) {
  const int J = g.kx * g.ky * g.kz;
  const int64_t sxy = (int64_t)g.nx * g.ny;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < J; c += gridDim.x * blockDim.x) {
    const int cx = c % g.kx, cy = (c / g.kx) % g.ky, cz = c / (g.kx * g.ky);
    const int lo[3] = {cx * C3, cy * C3, cz * C3};
    const int hi[3] = {cell_lo3(cx + 1, g.nx), cell_lo3(cy + 1, g.ny), cell_lo3(cz + 1, g.nz)};
    double sum = 0.0;
    int cnt = 0;
    for (int i = lo[0]; i < hi[0]; ++i) {
      double pl = 0.0;
      for (int j = lo[1]; j < hi[1]; ++j)
        for (int k = lo[2]; k < hi[2]; ++k) {
          const int64_t x = k * sxy + (int64_t)j * g.nx + i;
          if (g.mask && !g.mask[x]) continue;
          pl += g.F[x];
          cnt++;
        }
      sum += pl;
    }
    double Fc = cnt > 0 ? sum / cnt : 1.0;
    const int is0 = (lo[0] + hi[0] - 1) / 2, is1 = (lo[0] + hi[0]) / 2;
    const int js0 = (lo[1] + hi[1] - 1) / 2, js1 = (lo[1] + hi[1]) / 2;
    const int ks0 = (lo[2] + hi[2] - 1) / 2, ks1 = (lo[2] + hi[2]) / 2;
    double sc = 0.0;
    int nc = 0;
    for (int a = 0; a < (is0 == is1 ? 1 : 2); ++a)
      for (int b = 0; b < (js0 == js1 ? 1 : 2); ++b)
        for (int e = 0; e < (ks0 == ks1 ? 1 : 2); ++e) {
          const int64_t x = (e ? ks1 : ks0) * sxy + (int64_t)(b ? js1 : js0) * g.nx + (a ? is1 : is0);
          if (g.mask && !g.mask[x]) continue;
          sc += g.F[x];
          nc++;
        }
    if (nc > 0) Fc = sc / nc;
    const double q = f.cq[c];
    f.cacc[c] = cnt > 0;
    f.dc[c] = cnt > 0 ? f.hc / Fc : __builtin_huge_val();
    f.Uc[c] = q;  // +inf unless an exit cell
    f.lab[c] = 0;
    f.rank[c] = -1;
    f.level[c] = -1;
    if (q < __builtin_huge_val()) {
      const int slot = __hip_atomic_fetch_add(&f.ctl[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      f.srcs[slot] = c;
    }
  }
}

// Coarse exit cells by (q, index): the position of each is the number of
// cells before it.
__global__ void k3f_src_rank(Grid3 g, Fmsm3 f) {
  const int ns = f.ctl[0];
  for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < ns; a += gridDim.x * blockDim.x) {
    const int ca = f.srcs[a];
    const double qa = f.cq[ca];
    int r = 0;
    for (int b = 0; b < ns; ++b) {
      const int cb = f.srcs[b];
      const double qb = f.cq[cb];
      r += (qb < qa || (qb == qa && cb < ca)) ? 1 : 0;
    }
    f.sorted[r] = ca;
  }
}

// Fast Marching on the coarse grid (one wave), in the CPU oracle's order: the
// exit cells first, accepted together and then relaxed in (q, index) order;
// then the smallest (value, index) cell of the front, whose six neighbours
// are relaxed with the update from all six of their current neighbour values.
// The front is unordered in LDS; each acceptance is a wave-wide argmin.  The
// rank of a cell is its acceptance position, its level one more than the
// highest level among the neighbours accepted before it; accessible cells the
// front never reaches follow in index order.  LOCAL: the coarse values,
// states, levels and front positions live in LDS too (up to kLocal3 cells;
// the front then holds every cell), else in device memory with coherent
// accesses.
constexpr int kLocal3 = 4928;  // 32 bytes of LDS per cell

template <bool LOCAL>
struct FmmSmem;
template <>
struct FmmSmem<false> {
  double fv[kFront3];
  int32_t fi[kFront3];
};
template <>
struct FmmSmem<true> {
  double fv[kLocal3];
  double U[kLocal3];
  double dc[kLocal3];
  int16_t fi[kLocal3];
  int16_t lvl[kLocal3];
  int16_t pos[kLocal3];
  uint8_t lab[kLocal3];
  uint8_t acc[kLocal3];
};

template <bool LOCAL>
__global__ __launch_bounds__(64) void k3f_fmm(Grid3 g, Fmsm3 f) {
  __shared__ FmmSmem<LOCAL> sm;
  constexpr int CAP = LOCAL ? kLocal3 : kFront3;
  const int lane = threadIdx.x;
  if (ld_coh(g.err)) return;  // invalid input: reported by the host
  const int J = g.kx * g.ky * g.kz;
  const int ns = ld_coh(&f.ctl[0]);
  const double INF = __builtin_huge_val();
  // state accessors: LDS, or device memory; the kernel is one wave, the only
  // one that reads or writes this state while it runs, so workgroup-scope
  // accesses (cached by the compute unit) ordered by sync() suffice
  auto ldU = [&](int c) -> double {
    if constexpr (LOCAL) return sm.U[c]; else return ld_wg(&f.Uc[c]);
  };
  auto stU = [&](int c, double v) {
    if constexpr (LOCAL) sm.U[c] = v; else st_wg(&f.Uc[c], v);
  };
  auto ldLab = [&](int c) -> int {
    if constexpr (LOCAL) return sm.lab[c]; else return ld_wg(&f.lab[c]);
  };
  auto stLab = [&](int c, int v) {
    if constexpr (LOCAL) sm.lab[c] = (uint8_t)v; else st_wg(&f.lab[c], (uint8_t)v);
  };
  auto ldLvl = [&](int c) -> int {
    if constexpr (LOCAL) return sm.lvl[c]; else return ld_wg(&f.level[c]);
  };
  auto ldPos = [&](int c) -> int {
    if constexpr (LOCAL) return sm.pos[c]; else return ld_wg(&f.posf[c]);
  };
  auto stPos = [&](int c, int p) {
    if constexpr (LOCAL) sm.pos[c] = (int16_t)p; else st_wg(&f.posf[c], p);
  };
  auto sync = [&]() {
    if constexpr (LOCAL) {
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    } else {
      // the waits this needs for workgroup scope on this target come with the fence
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    }
  };
  auto ldDc = [&](int c) -> double {
    if constexpr (LOCAL) return sm.dc[c]; else return f.dc[c];
  };
  auto ldAcc = [&](int c) -> int {
    if constexpr (LOCAL) return sm.acc[c]; else return f.cacc[c];
  };
  if constexpr (LOCAL) {
    for (int c = lane; c < J; c += 64) {
      sm.U[c] = f.Uc[c];
      sm.dc[c] = f.dc[c];
      sm.acc[c] = f.cacc[c];
      sm.lab[c] = 0;
    }
    __syncthreads();
  }
  int maxlv = -1, na = 0, nf = 0;
  // cell c takes position na: rank, level (one more than the highest level
  // among its accepted neighbours), accepted
  auto place = [&](int c) {
    int lv = -1;
    if (lane < 6) {
      const int nb = nb_cell3(g, c, lane);
      if (nb >= 0 && ldLab(nb) == 2) lv = ldLvl(nb);
    }
    lv = wave_max_i(lv) + 1;
    if (lane == 0) {
      if constexpr (LOCAL) {
        sm.lvl[c] = (int16_t)lv;
        f.rank[c] = na;
        f.level[c] = lv;
      } else {
        st_wg(&f.rank[c], na);
        st_wg(&f.level[c], lv);
      }
      stLab(c, 2);
    }
    maxlv = lv > maxlv ? lv : maxlv;
    ++na;
    sync();
  };
  // relaxes the six neighbours of the accepted cell x (pairwise
  // non-adjacent: one lane each), every read of the step issued together;
  // PLACE: x is placed first (its level from the same reads); false when the
  // front would overflow
  auto relax = [&](int x, bool PLACE) -> bool {
    // coordinates once (no integer division per neighbour)
    const int xx = x % g.kx, xy = (x / g.kx) % g.ky, xz = x / (g.kx * g.ky);
    const int sy = g.kx, sz = g.kx * g.ky;
    const int ax = lane == 0 ? -1 : lane == 1 ? 1 : 0, ay = lane == 2 ? -1 : lane == 3 ? 1 : 0,
              az = lane == 4 ? -1 : lane == 5 ? 1 : 0;
    const int nx = xx + ax, ny = xy + ay, nz = xz + az;
    const bool nin = lane < 6 && nx >= 0 && ny >= 0 && nz >= 0 && nx < g.kx && ny < g.ky && nz < g.kz;
    const int nb = nin ? x + ax + ay * sy + az * sz : -1;
    const int nbs = nin ? nb : x;
    const int bx = nin ? nx : xx, by = nin ? ny : xy, bz = nin ? nz : xz;
    int mm[6];
    mm[0] = bx > 0 ? nbs - 1 : -1;
    mm[1] = bx + 1 < g.kx ? nbs + 1 : -1;
    mm[2] = by > 0 ? nbs - sy : -1;
    mm[3] = by + 1 < g.ky ? nbs + sy : -1;
    mm[4] = bz > 0 ? nbs - sz : -1;
    mm[5] = bz + 1 < g.kz ? nbs + sz : -1;
    const int ln = ldLab(nbs);
    const int lvn = ldLvl(nbs);
    const int an = ldAcc(nbs);
    const double dn = ldDc(nbs), un = ldU(nbs);
    const int pn = ldPos(nbs);
    double v[6];
    for (int e = 0; e < 6; ++e) v[e] = ldU(mm[e] >= 0 ? mm[e] : nbs);
    for (int e = 0; e < 6; ++e) v[e] = mm[e] >= 0 ? v[e] : INF;
    if (PLACE) {
      const int lv = wave_max_i(lane < 6 && nb >= 0 && ln == 2 ? lvn : -1) + 1;
      if (lane == 0) {
        if constexpr (LOCAL) {
          sm.lvl[x] = (int16_t)lv;
          f.rank[x] = na;
          f.level[x] = lv;
        } else {
          st_wg(&f.rank[x], na);
          st_wg(&f.level[x], lv);
        }
        stLab(x, 2);
      }
      maxlv = lv > maxlv ? lv : maxlv;
      ++na;
    }
    const bool live = lane < 6 && nb >= 0 && an && ln != 2;
    bool fresh = false;
    double u = un;
    if (live) {
      const double a = v[0] < v[1] ? v[0] : v[1], b = v[2] < v[3] ? v[2] : v[3],
                   cc = v[4] < v[5] ? v[4] : v[5];
      const double t = update3(a, b, cc, dn);
      if (t < u) {
        u = t;
        stU(nb, t);
      }
      if (ln == 0) {
        stLab(nb, 1);
        fresh = true;
      } else {
        sm.fv[pn] = u;
      }
    }
    const unsigned long long m = __ballot(fresh);
    const int add = __popcll(m);
    if (nf + add > CAP) return false;
    if (fresh) {
      const int p = nf + __popcll(m & ((1ull << lane) - 1ull));
      sm.fv[p] = u;
      sm.fi[p] = nb;
      stPos(nb, p);
    }
    nf += add;
    sync();
    return true;
  };
  bool ok = true;
  for (int s = 0; s < ns; ++s) place(f.sorted[s]);  // sources: accepted in (q, index) order ...
  for (int s = 0; s < ns && ok; ++s) ok = relax(f.sorted[s], false);  // ... then relaxed
  while (ok && nf > 0) {
    // the (value, index) minimum of the front; each lane takes four of its
    // slots per round so that their LDS reads are in flight together
    double bv = INF;
    int bi = 0x7fffffff, bp = -1;
    for (int t0 = lane; t0 < nf; t0 += 256) {
      int cq[4];
      double vq[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool in = t0 + 64 * k < nf;
        cq[k] = in ? (int)sm.fi[t0 + 64 * k] : 0;
        vq[k] = in ? sm.fv[t0 + 64 * k] : INF;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool take = t0 + 64 * k < nf && (vq[k] < bv || (vq[k] == bv && cq[k] < bi));
        bv = take ? vq[k] : bv;
        bi = take ? cq[k] : bi;
        bp = take ? t0 + 64 * k : bp;
      }
    }
    wave::argmin(bv, bi, bp, lane);
    if (lane == 0 && bp != nf - 1) {  // the last entry fills the hole
      sm.fv[bp] = sm.fv[nf - 1];
      sm.fi[bp] = sm.fi[nf - 1];
      stPos(sm.fi[bp], bp);
    }
    --nf;
    sync();
    ok = relax(bi, true);
  }
  if (!ok) {
    if (lane == 0) __hip_atomic_fetch_or(g.err, kErr3Front, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  // accessible cells the coarse front never reached, in index order
  for (int base = 0; base < J; base += 64) {
    const int c = base + lane;
    const bool left = c < J && ldAcc(c) && ldLab(c) != 2;
    unsigned long long m = __ballot(left);
    while (m) {
      const int k = __builtin_ctzll(m);
      m &= m - 1ull;
      place(base + k);
    }
  }
  if constexpr (LOCAL)
    for (int c = lane; c < J; c += 64) f.Uc[c] = sm.U[c];
  if (lane == 0) {
    st_coh(&f.ctl[1], maxlv + 1);
    st_coh(&f.ctl[2], na);
  }
}

// Part II for the cells of one level, one wave per cell: cells holding exit
// nodes and cells the coarse front never reached are swept to convergence
// cycling the orderings with the standard update; the others are swept once
// in each ordering their earlier neighbours allow, with the directional
// update.
__global__ __launch_bounds__(64) void k3f_level(Grid3 g, Fmsm3 f, int level) {
  __shared__ double tu[P3 * P3 * P3];
  __shared__ double td[C3 * C3 * C3];
  __shared__ uint8_t dec[C3 * C3 * C3];
  const int lane = threadIdx.x;
  const double INF = __builtin_huge_val();
  const int J = g.kx * g.ky * g.kz;
  const int64_t sxy = (int64_t)g.nx * g.ny;
  const int thin = (g.nx == 1 ? 1 : 0) | (g.ny == 1 ? 2 : 0) | (g.nz == 1 ? 4 : 0);
  unsigned long long nvis = 0, nsw = 0;
  for (int c = blockIdx.x; c < J; c += gridDim.x) {
    if (f.level[c] != level) continue;
    const int rc = f.rank[c];
    const bool conv = f.cq[c] < INF || f.Uc[c] == INF;
    int faces = 0;
    if (lane < 6) {
      const int nb = nb_cell3(g, c, lane);
      if (nb >= 0) {
        const int rn = f.rank[nb];
        if (rn >= 0 && rn < rc) faces = 1 << lane;
      }
    }
    for (int off = 32; off >= 1; off >>= 1) faces |= __shfl_xor(faces, off);
    const uint32_t mask = orderings3(faces, thin);
    const int cx = c % g.kx, cy = (c / g.kx) % g.ky, cz = c / (g.kx * g.ky);
    const int x0 = cx * C3, y0 = cy * C3, z0 = cz * C3;
    const int w = cell_lo3(cx + 1, g.nx) - x0, hg = cell_lo3(cy + 1, g.ny) - y0,
              dp = cell_lo3(cz + 1, g.nz) - z0;
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
    if (conv) {
      for (int sw = 0;; ++sw) {
        ++nsw;
        if (!sweep_cell3<false>(tu, td, dec, seq3(sw & 7), w, hg, dp, lane)) break;
        if (sw > 4096) {
          if (lane == 0) __hip_atomic_fetch_or(g.err, kErr3Guard, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    } else {
      for (int qq = 0; qq < 8; ++qq) {
        const int d = seq3(qq);
        if (!((mask >> d) & 1u)) continue;
        ++nsw;
        sweep_cell3<true>(tu, td, dec, d, w, hg, dp, lane);
      }
    }
    ++nvis;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ND; ++r) {
      const int t = lane + 64 * r;
      const int a = t % C3, b = (t / C3) % C3, e = t / (C3 * C3);
      if (a < w && b < hg && e < dp && dec[t])
        st_coh(g.u + (z0 + e) * sxy + (int64_t)(y0 + b) * g.nx + x0 + a,
               tu[((e + 1) * P3 + b + 1) * P3 + a + 1]);
    }
    __syncthreads();  // the next cell reuses the LDS arrays
  }
  if (lane == 0 && nvis) {
    __hip_atomic_fetch_add(&f.stats[0], nvis, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&f.stats[1], nsw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

hipError_t launch3_round(const Grid3& g, int round, int blocks, int cap, hipStream_t stream) {
  hipLaunchKernelGGL(k3_round, dim3(blocks), dim3(64), 0, stream, g, round, cap);
  return hipGetLastError();
}

hipError_t launch3f_prepare(const Grid3& g, const Fmsm3& f, hipStream_t stream) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const int J = g.kx * g.ky * g.kz;
  hipLaunchKernelGGL(k3_prep, dim3(grid_for3(n, 256, 8192)), dim3(256), 0, stream, g);
  hipLaunchKernelGGL(k3f_init, dim3(grid_for3(J, 256, 4096)), dim3(256), 0, stream, g, f);
  hipLaunchKernelGGL(k3f_sources, dim3(grid_for3(g.nsrc, 256, 1024)), dim3(256), 0, stream, g, f);
  hipLaunchKernelGGL(k3f_coarse, dim3(grid_for3(J, 64, 4096)), dim3(64), 0, stream, g, f);
  hipLaunchKernelGGL(k3f_src_rank, dim3(grid_for3(J, 256, 4096)), dim3(256), 0, stream, g, f);
  if (J <= kLocal3)
    hipLaunchKernelGGL(k3f_fmm<true>, dim3(1), dim3(64), 0, stream, g, f);
  else
    hipLaunchKernelGGL(k3f_fmm<false>, dim3(1), dim3(64), 0, stream, g, f);
  return hipGetLastError();
}

hipError_t launch3f_level(const Grid3& g, const Fmsm3& f, int level, int blocks, hipStream_t stream) {
  hipLaunchKernelGGL(k3f_level, dim3(blocks), dim3(64), 0, stream, g, f, level);
  return hipGetLastError();
}

int fmsm3_blocks_per_cu() {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void*>(k3f_level), 64, 0) !=
          hipSuccess || b < 1)
    b = 1;
  return b;
}

int round3_blocks_per_cu() {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void*>(k3_round), 64, 0) !=
          hipSuccess || b < 1)
    b = 1;
  return b;
}

}  // namespace eik
