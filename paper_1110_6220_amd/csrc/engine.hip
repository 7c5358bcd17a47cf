// HIP engine of libeik for gfx950 (MI355X).
//
// Method (Chacon & Vladimirsky, "Fast two-scale methods for Eikonal
// equations"): the grid is split into cells; a cell is processed by
// Gauss-Seidel sweeps over the cell with its one-node halo held fixed
// (Algorithm FSM restricted to c~ = c u N^f(c)); after processing, each
// neighbour cell is re-queued when a node on the shared side decreased during
// this processing (or is an exit node and the cell is removed for the first
// time) and is smaller than the node across (Algorithm generic_LC_cells).  The
// Theorem of Section 3.2.1 makes the result independent of the order in which
// cells are removed, which is what lets many cells run at once here.
//
// Mapping onto CDNA4:
//  * one wave64 per cell, cells up to 64 x 64 nodes; the tile plus its halo
//    and the per-node step delta = h/F live in LDS;
//  * a sweep walks the anti-diagonals of the tile: lane l owns column l and
//    at step d updates row d - l, so the upwind x-neighbour is the value lane
//    l-1 produced one step earlier, carried by a DPP wave shift, and the
//    upwind y-neighbour is the lane's own previous value -- the dependent
//    chain stays in registers; the two downwind neighbours are old values in
//    LDS.  This order is a topological order of the lexicographic sweep's
//    dependencies, so each sweep equals the serial sweep bit for bit;
//  * a persistent grid of waves pulls cells from a bucketed device queue
//    keyed by the cell values of eq. cell_value; state words per cell make
//    "queued", "running" and "re-queued while running" atomic transitions;
//  * values shared between waves (the solution array, cell states, queue)
//    use agent-scope atomics so that waves on different XCDs see each other's
//    writes; the read-only delta array uses ordinary cached loads.
#include <math.h>
#include <stdint.h>

#include "engine.h"

namespace eik {
namespace {


// ----------------------------------------------------------------------------
// scalar helpers
// ----------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T inf_v();
template <>
__device__ __forceinline__ double inf_v<double>() { return __builtin_huge_val(); }
template <>
__device__ __forceinline__ float inf_v<float>() { return __builtin_huge_valf(); }

template <typename T>
__device__ __forceinline__ T ld_coh(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_coh(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long ld64(const unsigned long long* p) {
  return ld_coh(p);
}

// Local update of Section 2 with the quadrant shortcut: a = min(U_W, U_E),
// b = min(U_S, U_N).  One-sided value min(a,b) + delta when |a - b| >= delta,
// otherwise the root >= max(a,b) of ((U-a)^2 + (U-b)^2) = delta^2.  The
// expression order matches the CPU oracle and the build disables contraction,
// so both round identically.
__device__ __forceinline__ double local_update(double a, double b, double dl) {
  const double lo = a < b ? a : b;
  const double d = a - b;
  const double one = lo + dl;
  const double two = 0.5 * (a + b + sqrt(2.0 * dl * dl - d * d));
  const double r = (fabs(d) >= dl) ? one : two;
  return (lo == __builtin_huge_val()) ? lo : r;
}

// FP32 storage: the branch test and the two-sided root are evaluated in FP64
// and rounded once to FP32.
__device__ __forceinline__ float local_update(float a, float b, float dl) {
  const float lo = a < b ? a : b;
  const double da = a, db = b, dd = da - db, ddl = dl;
  const float one = lo + dl;
  const float two = (float)(0.5 * (da + db + sqrt(2.0 * ddl * ddl - dd * dd)));
  const float r = (fabs(dd) >= ddl) ? one : two;
  return (lo == __builtin_huge_valf()) ? lo : r;
}

// Lane l receives lane l-1's value (DPP wave_shr:1; lane 0 receives 0).
__device__ __forceinline__ float wave_shr1(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ double wave_shr1(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x138, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int bcast(int v, int src_lane) { return __shfl(v, src_lane, 64); }

__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot(p); }

// orderable encoding of a float as an unsigned int (monotone)
__device__ __forceinline__ unsigned int key_bits(float f) {
  const unsigned int b = __builtin_bit_cast(unsigned int, f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key_float(unsigned int k) {
  const unsigned int b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __builtin_bit_cast(float, b);
}

__device__ __forceinline__ int cell_lo(int k, int n, int K, int s, int bal) {
  if (k >= K) return n;
  return bal ? (int)(((long long)k * n) / K) : k * s;
}

__device__ __forceinline__ const Inst& inst_of(const Engine& e, int g) {
  return e.ninst == 1 ? e.one : e.inst[e.cell_inst[g]];
}

__device__ __forceinline__ bool past_deadline(const Ctl* c) {
  return wall_clock64() > c->deadline;
}

__device__ __forceinline__ void set_err(Ctl* c, unsigned bits) {
  __hip_atomic_fetch_or(&c->err, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ----------------------------------------------------------------------------
// bucketed cell queue (per-lane operations)
// ----------------------------------------------------------------------------

__device__ __forceinline__ unsigned long long band_of(const Queue& q, float key) {
  if (q.nb <= 1 || !(key > 0.0f)) return 0;
  const double b = (double)key * q.inv_width;
  return b < 1e15 ? (unsigned long long)b : 1000000000000000ull;
}

// Appends `cell` to the ring of its band.  Every cell is in the queue at most
// once (guarded by its state word) and cap > cells, so a producer only waits
// for a consumer that has already claimed the slot's previous ticket.
__device__ bool q_push(const Engine& e, uint32_t cell, float key) {
  const Queue& q = e.q;
  uint32_t r = 0;
  if (q.nb > 1) {
    unsigned long long b = band_of(q, key);
    const unsigned long long cur = ld64(q.cursor);
    if (b < cur) b = cur;
    r = (uint32_t)(b & (q.nb - 1));
  }
  const unsigned long long t = __hip_atomic_fetch_add(
      &q.tail[r * kCtrStride], 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  unsigned long long* s = q.slot + (size_t)r * q.cap + (t & (q.cap - 1));
  while ((uint32_t)(ld64(s) >> 32) != (uint32_t)t) {
    if (past_deadline(e.ctl)) {
      set_err(e.ctl, kErrDeadline);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  __hip_atomic_store(s, ((t + 1ull) << 32) | cell, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// Wave-cooperative pop from the lowest non-empty band; -1 if none was found.
__device__ int q_pop(const Engine& e, int lane) {
  const Queue& q = e.q;
  unsigned long long cur = 0;
  if (q.nb > 1) cur = ld64(q.cursor);
  unsigned long long h = 0, t = 0;
  bool has = false;
  if ((uint32_t)lane < q.nb) {
    const uint32_t r = (uint32_t)((cur + lane) & (q.nb - 1));
    h = ld64(&q.head[r * kCtrStride]);
    t = ld64(&q.tail[r * kCtrStride]);
    has = h < t;
  }
  const unsigned long long m = ballot(has);
  if (!m) return -1;
  const int k = __builtin_ctzll(m);
  int cell = -1;
  if (lane == k) {
    const uint32_t r = (uint32_t)((cur + k) & (q.nb - 1));
    unsigned long long* hp = &q.head[r * kCtrStride];
    bool got = false;
    for (int tries = 0; tries < 8 && h < t; ++tries) {
      unsigned long long exp = h;
      if (__hip_atomic_compare_exchange_strong(hp, &exp, h + 1ull, __ATOMIC_RELAXED,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        got = true;
        break;
      }
      h = exp;
      t = ld64(&q.tail[r * kCtrStride]);
    }
    if (got) {
      unsigned long long* s = q.slot + (size_t)r * q.cap + (h & (q.cap - 1));
      unsigned long long v;
      for (;;) {
        v = __hip_atomic_load(s, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(v >> 32) == (uint32_t)(h + 1ull)) break;
        if (past_deadline(e.ctl)) {
          set_err(e.ctl, kErrDeadline);
          v = ~0ull;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (v != ~0ull) {
        cell = (int)(uint32_t)v;
        st_coh(s, (h + (unsigned long long)q.cap) << 32);
        if (k > 0) {
          unsigned long long c = cur;
          if (__hip_atomic_compare_exchange_strong(q.cursor, &c, cur + (unsigned long long)k,
                                                   __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT))
            __hip_atomic_fetch_add(&e.ctl->band_steps, 1ull, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  }
  return bcast(cell, k);
}

// Marks neighbour cell `g` as needing processing with direction flags `fl`;
// enqueues it when it was idle.  Called by one lane.
__device__ void requeue(const Engine& e, int g, uint32_t fl, float key) {
  const uint32_t old = __hip_atomic_fetch_or(&e.st[g], kPending | (fl << kFlagShift),
                                             __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  if (!(old & (kPending | kRunning))) {
    __hip_atomic_fetch_add(&e.ctl->active, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    q_push(e, (uint32_t)g, key);
  }
}

// ----------------------------------------------------------------------------
// the cell sweep
// ----------------------------------------------------------------------------

// One Gauss-Seidel sweep in direction dir (0 SW, 1 NW, 2 NE, 3 SE: x and y
// ascending for SW, x ascending / y descending for NW, ...) over the w x hgt
// tile in LDS (pitch P, halo at row/column 0 and w+1/hgt+1).  Returns whether
// any node decreased (wave-uniform).
template <typename T, int P>
__device__ bool sweep_tile(T* tu, const T* td, int w, int hgt, int dir, int lane) {
  const int sx = (dir == 0 || dir == 1) ? 1 : -1;
  const int sy = (dir == 0 || dir == 3) ? 1 : -1;
  const int i = sx > 0 ? lane : w - 1 - lane;
  const bool col_ok = lane < w;
  const int xoff = sx;        // step to the downwind x-neighbour in LDS
  const int yoff = sy * P;    // step to the downwind y-neighbour in LDS
  T prev = inf_v<T>();
  bool changed = false;
  const int nsteps = w + hgt - 1;
  for (int d = 0; d < nsteps; ++d) {
    const T from_left = wave_shr1(prev);
    const int t = d - lane;
    if (col_ok && t >= 0 && t < hgt) {
      const int j = sy > 0 ? t : hgt - 1 - t;
      const int idx = (j + 1) * P + (i + 1);
      const T wv = lane == 0 ? tu[idx - xoff] : from_left;
      const T sv = t == 0 ? tu[idx - yoff] : prev;
      const T ev = tu[idx + xoff];
      const T nv = tu[idx + yoff];
      const T uo = tu[idx];
      const T a = wv < ev ? wv : ev;
      const T b = sv < nv ? sv : nv;
      const T U = local_update(a, b, td[idx]);
      T r = uo;
      if (U < uo) {
        r = U;
        tu[idx] = U;
        changed = true;
      }
      prev = r;
    }
  }
  return ballot(changed) != 0ull;
}

// wave-wide max of x with the lowest lane attaining it (x = -inf: none)
__device__ __forceinline__ float wave_max(float x, int lane, int* arg) {
  float m = x;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const float y = __shfl_xor(m, o, 64);
    m = y > m ? y : m;
  }
  const unsigned long long at = ballot(x == m && m > -__builtin_huge_valf());
  *arg = at ? __builtin_ctzll(at) : -1;
  return m;
}

// ----------------------------------------------------------------------------
// persistent solver kernel
// ----------------------------------------------------------------------------

struct CellBox {
  int cx, cy, x0, x1, y0, y1, w, hgt;
};

__device__ __forceinline__ CellBox cell_box(const Inst& I, int local) {
  CellBox b;
  b.cx = local % I.kx;
  b.cy = local / I.kx;
  b.x0 = cell_lo(b.cx, I.nx, I.kx, I.s, I.balanced);
  b.x1 = cell_lo(b.cx + 1, I.nx, I.kx, I.s, I.balanced);
  b.y0 = cell_lo(b.cy, I.ny, I.ky, I.s, I.balanced);
  b.y1 = cell_lo(b.cy + 1, I.ny, I.ky, I.s, I.balanced);
  b.w = b.x1 - b.x0;
  b.hgt = b.y1 - b.y0;
  return b;
}

// Loads the tile (rows -1..hgt, columns -1..w without corners) from u and
// delta into LDS.  Outside the grid: +inf.
template <typename T, int P>
__device__ void load_tile(T* tu, T* td, const Inst& I, const CellBox& B, int lane,
                          bool with_interior) {
  const T* u = static_cast<const T*>(I.u);
  const T* dl = static_cast<const T*>(I.delta);
  const T INF = inf_v<T>();
  for (int r = -1; r <= B.hgt; ++r) {
    if (!with_interior && r >= 0 && r < B.hgt) continue;
    const int j = B.y0 + r;
    if (lane < B.w) {
      T v = INF, dv = INF;
      if (j >= 0 && j < I.ny) {
        const size_t k = (size_t)j * I.nx + B.x0 + lane;
        v = ld_coh(u + k);
        dv = dl[k];
      }
      tu[(r + 1) * P + lane + 1] = v;
      td[(r + 1) * P + lane + 1] = dv;
    }
  }
  if (lane < B.hgt) {
    const size_t row = (size_t)(B.y0 + lane) * I.nx;
    T vw = INF, dw = INF, ve = INF, de = INF;
    if (B.x0 > 0) {
      vw = ld_coh(u + row + B.x0 - 1);
      dw = dl[row + B.x0 - 1];
    }
    if (B.x1 < I.nx) {
      ve = ld_coh(u + row + B.x1);
      de = dl[row + B.x1];
    }
    tu[(lane + 1) * P] = vw;
    td[(lane + 1) * P] = dw;
    tu[(lane + 1) * P + B.w + 1] = ve;
    td[(lane + 1) * P + B.w + 1] = de;
  }
}

// Speed at y_i for eq. cell_value: at the node (integer offset) or the mean of
// the two straddling accessible nodes (half-integer offset); 0 = undefined.
template <typename T>
__device__ double speed_at(const Inst& I, int side, int along, int other, int wk) {
  const int dir = (side == 1 || side == 3) ? 1 : -1;
  const int twice = 2 * along + dir * (1 + wk);
  int p[2], np = 0;
  if ((twice & 1) == 0) {
    p[np++] = twice / 2;
  } else {
    p[np++] = (twice - 1) / 2;
    p[np++] = (twice - 1) / 2 + 1;
  }
  const T* F = static_cast<const T*>(I.F);
  double sum = 0.0;
  int cnt = 0;
  for (int m = 0; m < np; ++m) {
    const int ii = side <= 1 ? p[m] : other;
    const int jj = side <= 1 ? other : p[m];
    if (ii < 0 || jj < 0 || ii >= I.nx || jj >= I.ny) continue;
    const size_t k = (size_t)jj * I.nx + ii;
    if (I.mask && !I.mask[k]) continue;
    sum += (double)F[k];
    cnt++;
  }
  return cnt ? sum / cnt : 0.0;
}

// Directions raised in a receiving cell by a neighbour on its side s
// (0 W, 1 E, 2 S, 3 N): the two sweeps that start on that side.
__device__ __forceinline__ uint32_t side_dirs(int recv_side) {
  switch (recv_side) {
    case 0: return 0x1u | 0x2u;  // SW, NW
    case 1: return 0x4u | 0x8u;  // NE, SE
    case 2: return 0x1u | 0x8u;  // SW, SE
    default: return 0x2u | 0x4u; // NW, NE
  }
}

// After a sweep: writes the boundary nodes that decreased since they were
// last published, re-queues neighbours by the add criterion of Algorithm
// generic_LC_cells, and lowers their cell values (eq. cell_value).
template <typename T, int P>
__device__ void publish(const Engine& e, const Inst& I, const CellBox& B, int g, T* tu,
                        const T* td, T pub[4], bool first, int lane) {
  const T INF = inf_v<T>();
  T* u = static_cast<T*>(I.u);
  bool crit[4];
  float kv[4];
  int karg[4];
#pragma unroll
  for (int side = 0; side < 4; ++side) {
    // side 0 W: column 0, 1 E: column w-1 (lane = row); 2 S: row 0, 3 N: row
    // hgt-1 (lane = column)
    const bool vert = side <= 1;
    const int len = vert ? B.hgt : B.w;
    const bool ok = lane < len;
    int idx_in, idx_out;
    if (side == 0) { idx_in = (lane + 1) * P + 1; idx_out = idx_in - 1; }
    else if (side == 1) { idx_in = (lane + 1) * P + B.w; idx_out = idx_in + 1; }
    else if (side == 2) { idx_in = P + lane + 1; idx_out = idx_in - P; }
    else { idx_in = B.hgt * P + lane + 1; idx_out = idx_in + P; }
    bool c = false;
    float vmax = -__builtin_huge_valf();
    if (ok) {
      const T v = tu[idx_in];
      const bool is_src = td[idx_in] == INF && v != INF;
      const bool changed = v < pub[side] || (first && is_src);
      if (v < pub[side]) {
        const int ii = vert ? (side == 0 ? B.x0 : B.x1 - 1) : B.x0 + lane;
        const int jj = vert ? B.y0 + lane : (side == 2 ? B.y0 : B.y1 - 1);
        st_coh(u + (size_t)jj * I.nx + ii, v);
      }
      pub[side] = v;
      c = changed && td[idx_out] != INF && v < tu[idx_out];
      if (v != INF) vmax = (float)v;
    }
    crit[side] = ballot(c) != 0ull;
    kv[side] = wave_max(vmax, lane, &karg[side]);
  }
  // make the boundary values visible before any neighbour is signalled
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  if (lane < 4) {
    const int side = lane;
    int nb = -1, wk = 0;
    if (side == 0 && B.cx > 0) {
      nb = g - 1;
      wk = B.x0 - cell_lo(B.cx - 1, I.nx, I.kx, I.s, I.balanced);
    } else if (side == 1 && B.cx + 1 < I.kx) {
      nb = g + 1;
      wk = cell_lo(B.cx + 2, I.nx, I.kx, I.s, I.balanced) - B.x1;
    } else if (side == 2 && B.cy > 0) {
      nb = g - I.kx;
      wk = B.y0 - cell_lo(B.cy - 1, I.ny, I.ky, I.s, I.balanced);
    } else if (side == 3 && B.cy + 1 < I.ky) {
      nb = g + I.kx;
      wk = cell_lo(B.cy + 2, I.ny, I.ky, I.s, I.balanced) - B.y1;
    }
    if (nb >= 0) {
      float key = __builtin_huge_valf();
      if (karg[side] >= 0) {
        const int along = side == 0 ? B.x0 : side == 1 ? B.x1 - 1 : side == 2 ? B.y0 : B.y1 - 1;
        const int other = side <= 1 ? B.y0 + karg[side] : B.x0 + karg[side];
        const double fy = speed_at<T>(I, side, along, other, wk);
        if (fy > 0.0) {
          key = (float)((double)kv[side] + (0.5 * (1 + wk) * I.h) / fy);
          const unsigned int old =
              __hip_atomic_fetch_min(&e.key[nb], key_bits(key), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
          const float ok = key_float(old);
          if (ok < key) key = ok;
        }
      }
      if (crit[side]) {
        const int recv_side = side ^ 1;  // W<->E, S<->N
        requeue(e, nb, side_dirs(recv_side), key);
      }
    }
  }
}

template <typename T, int S>
__global__ __launch_bounds__(64) void k_solve(Engine e) {
  constexpr int P = S + 2;
  __shared__ T tu[P * P];
  __shared__ T td[P * P];
  const int lane = threadIdx.x;
  Ctl* ctl = e.ctl;
  if (__hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  int backoff = 0;
  for (;;) {
    const int g = q_pop(e, lane);
    if (g < 0) {
      const bool stop = ld64(&ctl->active) == 0ull ||
                        __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                        past_deadline(ctl);
      if (stop) break;
      if (backoff < 8) ++backoff;
      for (int z = 0; z < backoff; ++z) __builtin_amdgcn_s_sleep(2);
      continue;
    }
    backoff = 0;
    const Inst& I = inst_of(e, g);
    const CellBox B = cell_box(I, g - I.cell0);
    // claim the cell (acquire: halo values published before it was queued
    // are visible)
    uint32_t fl = 0;
    int first = 0;
    if (lane == 0) {
      const uint32_t old = __hip_atomic_exchange(&e.st[g], kRunning, __ATOMIC_ACQUIRE,
                                                 __HIP_MEMORY_SCOPE_AGENT);
      fl = (old >> kFlagShift) & 0xFu;
      const uint32_t v = ld_coh(&e.visits[g]);
      st_coh(&e.visits[g], v + 1u);
      first = v == 0u;
      const unsigned long long tot = __hip_atomic_fetch_add(&ctl->visits, 1ull, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
      if (tot >= ctl->guard) set_err(ctl, kErrGuard);
    }
    fl = (uint32_t)bcast((int)fl, 0);
    bool is_first = bcast(first, 0) != 0;
    load_tile<T, P>(tu, td, I, B, lane, true);
    T pub[4];
    pub[0] = lane < B.hgt ? tu[(lane + 1) * P + 1] : inf_v<T>();
    pub[1] = lane < B.hgt ? tu[(lane + 1) * P + B.w] : inf_v<T>();
    pub[2] = lane < B.w ? tu[P + lane + 1] : inf_v<T>();
    pub[3] = lane < B.w ? tu[B.hgt * P + lane + 1] : inf_v<T>();
    unsigned long long nsweeps = 0, nchecks = 0;
    int sched[4];
    for (;;) {
      // preferred directions first, in canonical order, then the others;
      // after four sweeps the canonical loop
      {
        int n = 0;
        for (int d = 0; d < 4; ++d)
          if (fl & (1u << d)) sched[n++] = d;
        for (int d = 0; d < 4; ++d)
          if (!(fl & (1u << d))) sched[n++] = d;
      }
      bool aborted = false;
      for (int k = 0;; ++k) {
        const int dir = k < 4 ? sched[k] : (k & 3);
        const bool ch = sweep_tile<T, P>(tu, td, B.w, B.hgt, dir, lane);
        if (ch) nsweeps++; else nchecks++;
        if (ch || is_first) {
          publish<T, P>(e, I, B, g, tu, td, pub, is_first, lane);
          is_first = false;
        }
        if (!ch) break;
        if (k > 4096) {  // a cell solve always terminates; guard anyway
          if (lane == 0) set_err(ctl, kErrGuard);
          aborted = true;
          break;
        }
      }
      if (aborted) break;
      // write the interior back (boundary nodes are already published)
      {
        T* u = static_cast<T*>(I.u);
        for (int r = 1; r + 1 < B.hgt; ++r)
          if (lane >= 1 && lane + 1 < B.w)
            st_coh(u + (size_t)(B.y0 + r) * I.nx + B.x0 + lane, tu[(r + 1) * P + lane + 1]);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      int again = 0;
      if (lane == 0) {
        uint32_t exp = kRunning;
        if (__hip_atomic_compare_exchange_strong(&e.st[g], &exp, 0u, __ATOMIC_RELEASE,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          __hip_atomic_fetch_add(&ctl->active, ~0ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
          // re-queued while running: take it again at once
          const uint32_t old = __hip_atomic_exchange(&e.st[g], kRunning, __ATOMIC_ACQUIRE,
                                                     __HIP_MEMORY_SCOPE_AGENT);
          fl = (old >> kFlagShift) & 0xFu;
          const uint32_t v = ld_coh(&e.visits[g]);
          st_coh(&e.visits[g], v + 1u);
          const unsigned long long tot = __hip_atomic_fetch_add(
              &ctl->visits, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (tot >= ctl->guard) set_err(ctl, kErrGuard);
          again = 1;
        }
      }
      again = bcast(again, 0);
      if (!again) break;
      if (__hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
      fl = (uint32_t)bcast((int)fl, 0);
      load_tile<T, P>(tu, td, I, B, lane, false);  // fresh halo only
    }
    if (lane == 0) {
      __hip_atomic_fetch_add(&ctl->sweeps, nsweeps, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&ctl->checks, nchecks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (__hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
  }
}

// ----------------------------------------------------------------------------
// preparation kernels
// ----------------------------------------------------------------------------

// Cell states, queue rings and control block.
__global__ void k_prep_cells(Engine e) {
  const int ninst = e.ninst;
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t c = tid; c < (size_t)e.ncells; c += stride) {
    e.st[c] = 0u;
    e.visits[c] = 0u;
    e.key[c] = 0xFF800000u;  // key_bits(+inf)
  }
  if (ninst > 1) {
    // instance of every cell (instances are laid out by increasing cell0)
    for (size_t c = tid; c < (size_t)e.ncells; c += stride) {
      int lo = 0, hi = ninst - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (e.inst[mid].cell0 <= (int)c) lo = mid; else hi = mid - 1;
      }
      e.cell_inst[c] = lo;
    }
  }
  const size_t nslot = (size_t)e.q.cap * e.q.nb;
  for (size_t k = tid; k < nslot; k += stride)
    e.q.slot[k] = (unsigned long long)(k & (e.q.cap - 1)) << 32;
  for (size_t k = tid; k < (size_t)e.q.nb; k += stride) {
    e.q.head[k * kCtrStride] = 0ull;
    e.q.tail[k * kCtrStride] = 0ull;
  }
  if (tid == 0) {
    *e.q.cursor = 0ull;
    Ctl* c = e.ctl;
    c->guard = e.guard;
    c->deadline = wall_clock64() + e.timeout_ticks;
    c->active = 0ull;
    c->visits = 0ull;
    c->sweeps = 0ull;
    c->checks = 0ull;
    c->band_steps = 0ull;
    c->mon_checks = 0ull;
    c->mon_ok = 0ull;
    c->resid_bits = 0ull;
    c->err = 0u;
    c->done_waves = 0u;
  }
}

// delta = h/F on accessible nodes (validating F), +inf on obstacles.
template <typename T>
__global__ void k_prep_nodes(Engine e) {
  const Inst& I = e.ninst == 1 ? e.one : e.inst[blockIdx.y];
  const size_t n = (size_t)I.nx * I.ny;
  const T* F = static_cast<const T*>(I.F);
  T* dl = static_cast<T*>(I.delta);
  bool bad = false;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x) {
    const bool acc = I.mask ? I.mask[k] != 0 : true;
    T d = inf_v<T>();
    if (acc) {
      const double f = (double)F[k];
      if (!(f > 0.0) || !isfinite(f)) bad = true;
      d = (T)(I.h / f);
    }
    dl[k] = d;
  }
  if (bad) set_err(e.ctl, kErrSpeed);
}

// Source validation (index range, accessibility, finite q).
__global__ void k_check_sources(Engine e) {
  const Inst& I = e.ninst == 1 ? e.one : e.inst[blockIdx.y];
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < I.nsrc; s += gridDim.x * blockDim.x) {
    const long long k = I.src[s];
    const double q = I.q ? I.q[s] : 0.0;
    const long long n = (long long)I.nx * I.ny;
    if (k < 0 || k >= n || (I.mask && !I.mask[k]) || !isfinite(q)) set_err(e.ctl, kErrSource);
  }
}

template <typename T>
__global__ void k_init_u(Engine e) {
  if (__hip_atomic_load(&e.ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const Inst& I = e.ninst == 1 ? e.one : e.inst[blockIdx.y];
  const size_t n = (size_t)I.nx * I.ny;
  T* u = static_cast<T*>(I.u);
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x)
    u[k] = inf_v<T>();
}

__device__ __forceinline__ void atomic_min_val(double* p, double v) {
  unsigned long long* a = reinterpret_cast<unsigned long long*>(p);
  unsigned long long old = *a;
  while (__builtin_bit_cast(double, old) > v) {
    if (__hip_atomic_compare_exchange_strong(a, &old, __builtin_bit_cast(unsigned long long, v),
                                             __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      break;
  }
}
__device__ __forceinline__ void atomic_min_val(float* p, float v) {
  unsigned int* a = reinterpret_cast<unsigned int*>(p);
  unsigned int old = *a;
  while (__builtin_bit_cast(float, old) > v) {
    if (__hip_atomic_compare_exchange_strong(a, &old, __builtin_bit_cast(unsigned int, v),
                                             __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      break;
  }
}

// u = min q at sources, sources frozen (delta = +inf), their cells queued
// (Algorithm generic_LC_cells, cell and fine-grid initialisation).
template <typename T>
__global__ void k_apply_sources(Engine e) {
  if (__hip_atomic_load(&e.ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const Inst& I = e.ninst == 1 ? e.one : e.inst[blockIdx.y];
  T* u = static_cast<T*>(I.u);
  T* dl = static_cast<T*>(I.delta);
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < I.nsrc; s += gridDim.x * blockDim.x) {
    const long long k = I.src[s];
    const double q = I.q ? I.q[s] : 0.0;
    atomic_min_val(u + k, (T)q);
    dl[k] = inf_v<T>();
    const int i = (int)(k % I.nx), j = (int)(k / I.nx);
    // cell containing (i, j)
    int cx = 0, cy = 0;
    while (cx + 1 < I.kx && cell_lo(cx + 1, I.nx, I.kx, I.s, I.balanced) <= i) cx++;
    while (cy + 1 < I.ky && cell_lo(cy + 1, I.ny, I.ky, I.s, I.balanced) <= j) cy++;
    const int g = I.cell0 + cy * I.kx + cx;
    const float key = e.method == kFhcm ? 0.0f : (float)q;
    __hip_atomic_fetch_min(&e.key[g], key_bits(key), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t fl = e.method == kFhcm ? 0xFu : 0u;
    requeue(e, g, fl, key);
  }
}

// Fixed-point residual max |T(u)_k - u_k| / u_k in FP64 over accessible,
// non-source nodes with finite u (inf where u is inf but T(u) is finite).
template <typename T>
__global__ void k_residual(Engine e) {
  const Inst& I = e.ninst == 1 ? e.one : e.inst[blockIdx.y];
  const T* u = static_cast<const T*>(I.u);
  const T* F = static_cast<const T*>(I.F);
  const T* dl = static_cast<const T*>(I.delta);
  const size_t n = (size_t)I.nx * I.ny;
  double mx = 0.0;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x) {
    if (dl[k] == inf_v<T>()) continue;  // obstacle or source
    const int i = (int)(k % I.nx), j = (int)(k / I.nx);
    const double INF = __builtin_huge_val();
    const double uW = i > 0 ? (double)u[k - 1] : INF;
    const double uE = i + 1 < I.nx ? (double)u[k + 1] : INF;
    const double uS = j > 0 ? (double)u[k - I.nx] : INF;
    const double uN = j + 1 < I.ny ? (double)u[k + I.nx] : INF;
    const double a = uW < uE ? uW : uE, b = uS < uN ? uS : uN;
    const double t = local_update(a, b, I.h / (double)F[k]);
    const double v = (double)u[k];
    double r;
    if (v == INF) r = (t == INF) ? 0.0 : INF;
    else r = fabs(t - v) / v;
    if (r > mx) mx = r;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    const double y = __shfl_xor(mx, o, 64);
    mx = y > mx ? y : mx;
  }
  if ((threadIdx.x & 63) == 0 && mx > 0.0)
    __hip_atomic_fetch_max(&e.ctl->resid_bits, __builtin_bit_cast(unsigned long long, mx),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------

static int grid_for(int64_t n, int block, int cap) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

hipError_t launch_prepare(const Engine& e, int64_t max_nodes, hipStream_t stream) {
  const int gy = e.ninst;
  const int64_t cwork = (int64_t)e.ncells > (int64_t)e.q.cap * e.q.nb
                            ? (int64_t)e.ncells : (int64_t)e.q.cap * e.q.nb;
  hipLaunchKernelGGL(k_prep_cells, dim3(grid_for(cwork, 256, 4096)), dim3(256), 0, stream, e);
  const dim3 gn(grid_for(max_nodes, 256, gy > 1 ? 512 : 8192), gy);
  if (e.dtype == 0) hipLaunchKernelGGL(k_prep_nodes<double>, gn, dim3(256), 0, stream, e);
  else hipLaunchKernelGGL(k_prep_nodes<float>, gn, dim3(256), 0, stream, e);
  hipLaunchKernelGGL(k_check_sources, dim3(1, gy), dim3(64), 0, stream, e);
  if (e.dtype == 0) hipLaunchKernelGGL(k_init_u<double>, gn, dim3(256), 0, stream, e);
  else hipLaunchKernelGGL(k_init_u<float>, gn, dim3(256), 0, stream, e);
  if (e.dtype == 0) hipLaunchKernelGGL(k_apply_sources<double>, dim3(1, gy), dim3(64), 0, stream, e);
  else hipLaunchKernelGGL(k_apply_sources<float>, dim3(1, gy), dim3(64), 0, stream, e);
  return hipGetLastError();
}

size_t solve_lds_bytes(int dtype, int tile) {
  const size_t P = (size_t)tile + 2;
  return 2 * P * P * (dtype == 0 ? sizeof(double) : sizeof(float));
}

hipError_t launch_solve(const Engine& e, int workers, int tile, hipStream_t stream) {
  const dim3 g(workers), b(64);
  if (e.dtype == 0) {
    if (tile <= 16) hipLaunchKernelGGL((k_solve<double, 16>), g, b, 0, stream, e);
    else if (tile <= 32) hipLaunchKernelGGL((k_solve<double, 32>), g, b, 0, stream, e);
    else hipLaunchKernelGGL((k_solve<double, 64>), g, b, 0, stream, e);
  } else {
    if (tile <= 16) hipLaunchKernelGGL((k_solve<float, 16>), g, b, 0, stream, e);
    else if (tile <= 32) hipLaunchKernelGGL((k_solve<float, 32>), g, b, 0, stream, e);
    else hipLaunchKernelGGL((k_solve<float, 64>), g, b, 0, stream, e);
  }
  return hipGetLastError();
}

hipError_t launch_residual(const Engine& e, int64_t max_nodes, hipStream_t stream) {
  const dim3 gn(grid_for(max_nodes, 256, e.ninst > 1 ? 256 : 4096), e.ninst);
  if (e.dtype == 0) hipLaunchKernelGGL(k_residual<double>, gn, dim3(256), 0, stream, e);
  else hipLaunchKernelGGL(k_residual<float>, gn, dim3(256), 0, stream, e);
  return hipGetLastError();
}

}  // namespace eik
