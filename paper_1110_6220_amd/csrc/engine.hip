// HIP engine of libeik for gfx950 (MI355X).
//
// Method (Chacon & Vladimirsky, "Fast two-scale methods for Eikonal
// equations"): the grid is split into cells; a cell is processed by
// Gauss-Seidel sweeps over the cell with its one-node halo held fixed
// (Algorithm FSM restricted to c~ = c u N^f(c)); after processing, a
// neighbour cell is re-queued when a node on the shared side decreased during
// this processing (or is an exit node and the cell is removed for the first
// time) and is smaller than the node across (Algorithm generic_LC_cells).  The
// Theorem of Section 3.2.1 makes the exact method's result independent of the
// order in which cells are removed, which is what lets many cells run at once.
//
// Mapping onto CDNA4:
//  * one wave64 per cell, cells up to 64 x 64 nodes; the tile, its halo and
//    the per-node step delta = h/F live in LDS;
//  * a sweep walks the anti-diagonals of the tile: lane l owns column l and
//    at step d updates row d - l, so the upwind x-neighbour is the value lane
//    l-1 produced one step earlier, carried by a DPP wave shift, and the
//    upwind y-neighbour is the lane's own previous value -- the dependent
//    chain stays in registers; downwind neighbours are old values in LDS.
//    This order is a topological order of the lexicographic sweep's
//    dependencies, so each sweep equals the serial sweep bit for bit;
//  * a persistent grid of waves pulls cells from a device queue.  Cells are
//    ordered either by the cell values of eq. cell_value in bands (the
//    Heap-Cell Methods' heap, relaxed to "any cell of the lowest open bands")
//    or, when a coarse solve is available (FMSM Part I), by dependency
//    counts: a cell starts once every neighbour that precedes it in the
//    coarse order has finished its first processing.  State words make
//    "queued", "running", "re-queued while running" and "first pass done"
//    atomic transitions;
//  * values shared between waves (solution, cell states, queue, counters)
//    use agent-scope atomics, coherent across XCDs; the read-only delta and
//    speed arrays use ordinary cached loads.
#include <math.h>
#include <stdint.h>

#include "engine.h"
#include "wave.h"


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

// Pointers into device global memory (address space 1): loads through them
// are global_load rather than flat_load.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> to_global(T* p) {
  return (gptr<T>)(p);
}

template <typename T>
__device__ __forceinline__ T ld_coh(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_coh(gptr<const T> p) {
  return __hip_atomic_load((gptr<T>)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_coh(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld64(const unsigned long long* p) {
  return ld_coh(p);
}

template <typename T>
__device__ __forceinline__ T atomic_add_relaxed(T* p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Square root of x >= 2^-767 by the reciprocal-square-root estimate and two
// Newton corrections (the sequence LLVM emits for a correctly rounded sqrt,
// without its rescaling of tiny inputs, which never occur here: the argument
// 2 delta^2 - d^2 is either >= delta^2 or the result is discarded).
__device__ __forceinline__ double sqrt_pos(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  double g = x * r;
  double h = r * 0.5;
  const double e = fma(-h, g, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
}

// The same root without the last correction: within one unit in the last
// place instead of correctly rounded, two dependent operations shorter.
__device__ __forceinline__ double sqrt_pos_faithful(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  double g = x * r;
  double h = r * 0.5;
  const double e = fma(-h, g, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  const double d = fma(-g, g, x);
  return fma(d, h, g);
}

template <bool FAITHFUL>
__device__ __forceinline__ double root_pos(double x) {
  if constexpr (FAITHFUL) return sqrt_pos_faithful(x);
  else return sqrt_pos(x);
}

// Local update of Section 2 from a (x-neighbour value) and b (y-neighbour
// value): the one-sided value min(a,b) + delta when |a - b| >= delta,
// otherwise the root >= max(a,b) of (U-a)^2 + (U-b)^2 = delta^2.  The
// two-sided value rounds exactly as the CPU oracle's 0.5 * ((a + b) + s): the
// fused 0.5 * s + 0.5 * (a + b) is that sum halved before its one rounding,
// and halving commutes with rounding (no operand is near the underflow
// range).  Contraction is otherwise off, so the remaining terms round as in
// the oracle too.  a = b = +inf gives NaN, which the caller's minimum with the
// old value turns into "no update".
// FAITHFUL (the exact method, whose bar is a relative error against the
// oracle, not bit equality): the discriminant as one fma and the root within
// one unit in the last place.
template <bool FAITHFUL = false>
__device__ __forceinline__ double local_update(double a, double b, double dl) {
  const double lo = wave::vmin(a, b);  // a and b are never NaN
  const double d = a - b;
  const double one = lo + dl;
  const double x = FAITHFUL ? fma(-d, d, 2.0 * dl * dl) : 2.0 * dl * dl - d * d;
  const double two = fma(0.5, root_pos<FAITHFUL>(x), 0.5 * (a + b));
  return (fabs(d) >= dl) ? one : two;
}

// FP32 storage: the branch test and the two-sided root are evaluated in FP64
// and rounded once to FP32.
template <bool FAITHFUL = false>
__device__ __forceinline__ float local_update(float a, float b, float dl) {
  const float lo = wave::vmin(a, b);
  const double da = a, db = b, dd = da - db, ddl = dl;
  const float one = lo + dl;
  const double x = FAITHFUL ? fma(-dd, dd, 2.0 * ddl * ddl) : 2.0 * ddl * ddl - dd * dd;
  const float two = (float)fma(0.5, root_pos<FAITHFUL>(x), 0.5 * (da + db));
  return (fabs(dd) >= ddl) ? one : two;
}

using wave::vmin;  // IEEE minNum without NaN canonicalisation (wave.h)

// Lane l receives lane l-1's value; lane 0 receives `edge` (DPP wave_shr:1
// with the out-of-range source replaced by the old value).
__device__ __forceinline__ float shr1_or(float v, float edge) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                               __builtin_bit_cast(int, v), 0x138,
                                                               0xf, 0xf, false));
}
__device__ __forceinline__ double shr1_or(double v, double edge) {
  const long long b = __builtin_bit_cast(long long, v);
  const long long o = __builtin_bit_cast(long long, edge);
  const int lo = __builtin_amdgcn_update_dpp((int)o, (int)b, 0x138, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), 0x138, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Broadcast of lane src_lane's value; the result is marked wave-uniform so
// that everything derived from it lives in scalar registers.
__device__ __forceinline__ int bcast(int v, int src_lane) {
  return __builtin_amdgcn_readfirstlane(__shfl(v, src_lane, 64));
}

// The lane id as a value the compiler cannot see through.  Each phase of a
// cell's processing (load, sweeps, publish, store) derives its addresses from
// its own opaque copy, so lane-derived values are computed where they are
// used instead of being hoisted and held in registers across other phases.
__device__ __forceinline__ int opaque_lane(int lane) {
  asm volatile("" : "+v"(lane));
  return lane;
}
__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot(p); }

// Orderable encoding of a cell value (a double, never NaN) as a 64-bit
// unsigned integer: a < b exactly when key_bits(a) < key_bits(b), so an
// integer atomic minimum keeps the smallest value exactly (eq. cell_value's
// estimates are compared in the precision they are computed in).
constexpr unsigned long long kKeyInf = 0xFFF0000000000000ull;  // key_bits(+inf)
constexpr unsigned long long kKeyNone = ~0ull;                 // above every value
__device__ __forceinline__ unsigned long long key_bits(double f) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, f);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double key_value(unsigned long long k) {
  const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __builtin_bit_cast(double, b);
}

__device__ __forceinline__ int cell_lo(int k, int n, int K, int s, int bal) {
  if (k >= K) return n;
  return bal ? (int)(((long long)k * n) / K) : k * s;
}

__device__ __forceinline__ int inst_index(const Engine& e, int g) {
  return e.ninst == 1 ? 0 : e.cell_inst[g];
}
__device__ __forceinline__ Inst inst_of(const Engine& e, int g) {
  return e.args_inst ? e.one : e.inst[inst_index(e, g)];
}

__device__ __forceinline__ bool past_deadline(const Ctl* c) {
  return wall_clock64() > c->deadline;
}

__device__ __forceinline__ void set_err(Ctl* c, unsigned bits) {
  __hip_atomic_fetch_or(&c->err, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned get_err(const Ctl* c) {
  return __hip_atomic_load(const_cast<unsigned*>(&c->err), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Profiling phases of a wave's time, summed in registers and added to the
// control block's t_idle .. t_finish once when the wave leaves.  Compiled in
// only with -DEIK_PROFILING (the sums cost registers); then EIK_PROFILE=1
// switches them on.
enum Phase { kPhIdle, kPhClaim, kPhLoad, kPhSweep, kPhPublish, kPhFinish, kPhases };
#ifdef EIK_PROFILING
constexpr bool kProfiling = true;
#else
constexpr bool kProfiling = false;
#endif

// Adds the ticks since *t0 to phase k (when profiling) and restarts the clock.
__device__ __forceinline__ void tick(const Engine& e, unsigned long long* ph, int k,
                                     unsigned long long* t0) {
  if constexpr (kProfiling) {
    if (!e.profile) return;
    const unsigned long long t = wall_clock64();
    ph[k] += t - *t0;
    *t0 = t;
  }
}

// Ordering between waves.  Every value the waves share (solution values,
// cell states, queue words, counters) is accessed only with agent-scope
// atomic operations, which are coherent across XCDs on their own; what the
// protocol needs on top is that a wave's earlier memory operations have
// completed before it signals (release) and that its later operations start
// after the signal it observed has returned (acquire).  Waiting on the
// wave's memory counters gives exactly that.  EIK_FENCE_MODE=1 uses the
// compiler's agent-scope fences instead, which in addition write back and
// invalidate the L2 for non-atomic data this kernel does not share.
#ifndef EIK_FENCE_MODE
#define EIK_FENCE_MODE 0
#endif
__device__ __forceinline__ void order_release() {
#if EIK_FENCE_MODE == 1
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
#else
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
#endif
}
__device__ __forceinline__ void order_acquire() {
#if EIK_FENCE_MODE == 1
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
#else
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
#endif
}

// ----------------------------------------------------------------------------
// cell queue (per-lane operations except q_pop)
// ----------------------------------------------------------------------------

__device__ __forceinline__ unsigned long long* ctr(unsigned long long* base, uint32_t r) {
  return base + (size_t)r * kCtrStride;
}

// The rings of one group: the whole queue (ng = 1) or one problem's.
// Counter index of the group's ring r: base + r.
struct QView {
  unsigned long long* slot;
  unsigned long long* cursor;
  uint32_t cap, base;
  double inv_width;
};
__device__ __forceinline__ QView qview(const Queue& q, uint32_t g) {
  if (q.ng <= 1) return QView{q.slot, q.cursor, q.cap, 0u, q.inv_width};
  const QGroup G = q.grp[g];
  return QView{q.slot + G.off, q.cursor + (size_t)g * kCtrStride, G.cap, g * q.nb, G.inv_width};
}

__device__ __forceinline__ unsigned long long band_of(const Queue& q, const QView& v, double key) {
  if (q.nb <= 1 || !(key > 0.0)) return 0;
  const double b = key * v.inv_width;
  return b < 1e15 ? (unsigned long long)b : 1000000000000000ull;
}

// Appends `cell` to the ring of its band (clamped to the open bands
// [cursor, cursor + nb)) in its problem's group.  Every cell is in the queue
// at most once (guarded by its state word) and cap > cells of the group, so a
// producer only waits for a consumer that has already claimed the slot's
// previous ticket.
// RINGS = false: the caller knows the FIFO has one ring (the single-problem
// solver, which thus carries none of the ring arithmetic).
template <bool RINGS = true>
__device__ void q_push(const Engine& e, uint32_t cell, double key) {
  const Queue& q = e.q;
  const QView v = qview(q, q.ng > 1 ? (uint32_t)e.cell_inst[cell] : 0u);
  uint32_t r = RINGS && q.nb == 1 ? cell & (q.nring - 1u) : 0u;
  if (q.nb > 1) {
    const unsigned long long kb = band_of(q, v, key);
    for (;;) {
      const unsigned long long c = ld64(v.cursor);
      unsigned long long b = kb < c ? c : kb;
      if (b > c + q.nb - 1) b = c + q.nb - 1;
      r = (uint32_t)(b & (q.nb - 1));
      const unsigned long long old = atomic_add_relaxed(ctr(q.inflight, v.base + r), 1ull);
      order_acquire();
      // band b still open and not yet passed by the cursor: the count now
      // held keeps the cursor from passing it
      if (!(old & kClosed) && ld64(v.cursor) <= b) break;
      atomic_add_relaxed(ctr(q.inflight, v.base + r), ~0ull);
      if (past_deadline(e.ctl)) {
        set_err(e.ctl, kErrDeadline);
        return;
      }
    }
    order_release();
  }
  const unsigned long long t = atomic_add_relaxed(ctr(q.tail, v.base + r), 1ull);
  unsigned long long* s = v.slot + (size_t)r * v.cap + (t & (v.cap - 1));
  // on the ring's first lap every slot is free
  while (t >= v.cap && (uint32_t)(ld64(s) >> 32) != (uint32_t)t) {
    if (past_deadline(e.ctl)) {
      set_err(e.ctl, kErrDeadline);
      return;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  order_release();
  st_coh(s, ((t + 1ull) << 32) | cell);
  if (q.ng > 1) atomic_add_relaxed(q.queued + (size_t)(v.base / q.nb) * kCtrStride, 1ull);
}

// Moves a group's cursor past its band c when no cell of that band is queued
// or running.  One lane.
__device__ void q_advance(const Engine& e, const QView& v, unsigned long long c) {
  const Queue& q = e.q;
  unsigned long long* fl = ctr(q.inflight, v.base + (uint32_t)(c & (q.nb - 1)));
  unsigned long long z = 0ull;
  if (!__hip_atomic_compare_exchange_strong(fl, &z, kClosed, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT))
    return;
  order_acquire();
  unsigned long long cc = c;
  const bool moved = __hip_atomic_compare_exchange_strong(v.cursor, &cc, c + 1ull, __ATOMIC_RELAXED,
                                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  order_release();
  __hip_atomic_fetch_and(fl, ~kClosed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (moved) atomic_add_relaxed(&e.ctl->band_steps, 1ull);
}

// Takes the cell at ticket h of counter ring r (group ring r - v.base) if
// the head is still there (a few retries while h < t).  One lane; -1 if
// nothing was taken.
__device__ int q_take(const Engine& e, const QView& v, uint32_t r, unsigned long long h,
                      unsigned long long t) {
  const Queue& q = e.q;
  unsigned long long* hp = ctr(q.head, r);
  bool got = false;
  for (int tries = 0; tries < 8 && h < t; ++tries) {
    unsigned long long exp = h;
    if (__hip_atomic_compare_exchange_strong(hp, &exp, h + 1ull, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      got = true;
      break;
    }
    h = exp;
    t = ld64(ctr(q.tail, r));
  }
  if (!got) return -1;
  unsigned long long* s = v.slot + (size_t)(r - v.base) * v.cap + (h & (v.cap - 1));
  unsigned long long w;
  for (;;) {
    w = ld64(s);
    if ((uint32_t)(w >> 32) == (uint32_t)(h + 1ull)) break;
    if (past_deadline(e.ctl)) {
      set_err(e.ctl, kErrDeadline);
      return -1;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  st_coh(s, (h + (unsigned long long)v.cap) << 32);
  return (int)(uint32_t)w;
}

// Wave-cooperative pop from the lowest non-empty band within the window;
// returns the cell (or -1) and its counter ring in *ring.
__device__ int q_pop(const Engine& e, int lane, int* ring) {
  const Queue& q = e.q;
  const QView v = qview(q, 0u);
  const unsigned long long cur = ld64(v.cursor);
  unsigned long long h = 0, t = 0;
  bool has = false;
  if ((uint32_t)lane <= q.window) {
    const uint32_t r = (uint32_t)((cur + lane) & (q.nb - 1));
    h = ld64(ctr(q.head, r));
    t = ld64(ctr(q.tail, r));
    has = h < t;
  }
  const unsigned long long m = ballot(has);
  if (!m) {
    if (lane == 0) q_advance(e, v, cur);
    return -1;
  }
  const int k = __builtin_ctzll(m);
  const uint32_t r = (uint32_t)((cur + k) & (q.nb - 1));
  int cell = -1;
  if (lane == k) cell = q_take(e, v, r, h, t);
  *ring = (int)r;
  return bcast(cell, k);
}

// Pop with one group per problem: lane l looks at group home + l (then
// home + 64 + l, ...).  A group with cells queued: the lowest non-empty band
// of its window, or, with the window empty, its cursor moves on; the first
// lane that found a cell takes it.  Returns the cell (or -1) and its counter
// ring.  The queued counts only steer the scan: a count read too low delays a
// cell to a later scan, one read too high costs a look at the group.
__device__ int q_pop_groups(const Engine& e, int lane, uint32_t home, int* ring) {
  const Queue& q = e.q;
  for (uint32_t base = 0; base < q.ng; base += 64u) {
    const uint32_t gi = base + (uint32_t)lane;
    bool has = false;
    uint32_t g = 0, r = 0;
    unsigned long long h = 0, t = 0;
    if (gi < q.ng) {
      g = home + gi;
      if (g >= q.ng) g -= q.ng;
    }
    if (gi < q.ng && ld64(q.queued + (size_t)g * kCtrStride) != 0ull) {
      const QView v = qview(q, g);
      const unsigned long long cur = ld64(v.cursor);
      for (uint32_t w = 0; w <= q.window; ++w) {
        r = v.base + (uint32_t)((cur + w) & (q.nb - 1));
        h = ld64(ctr(q.head, r));
        t = ld64(ctr(q.tail, r));
        if (h < t) {
          has = true;
          break;
        }
      }
      if (!has && ld64(ctr(q.inflight, v.base + (uint32_t)(cur & (q.nb - 1)))) == 0ull)
        q_advance(e, v, cur);
    }
    const unsigned long long m = ballot(has);
    if (!m) continue;
    const int k = __builtin_ctzll(m);
    int cell = -1;
    if (lane == k) {
      cell = q_take(e, qview(q, g), r, h, t);
      if (cell >= 0) atomic_add_relaxed(q.queued + (size_t)g * kCtrStride, ~0ull);
    }
    *ring = bcast((int)r, k);
    return bcast(cell, k);
  }
  return -1;
}

// Blocking pop from a single FIFO ring (nb = 1).  The wave takes the next
// ticket and waits on that ticket's slot only, so idle waves poll distinct
// addresses instead of competing for the head.  Returns the cell, or -1 once
// no cell is waiting, queued or running (or on error/timeout).  A ticket is
// given up only then: no cell will be queued any more.
template <bool RINGS>
__device__ int q_pop_ticket(const Engine& e, int lane, uint32_t ring) {
  const Queue& q = e.q;
  int cell = -1;
  if (!RINGS) ring = 0u;
  if (lane == 0) {
    const unsigned long long h = atomic_add_relaxed(ctr(q.head, ring), 1ull);
    unsigned long long* s = q.slot + (size_t)ring * q.cap + (h & (q.cap - 1));
    int spins = 0;
    for (;;) {
      const unsigned long long v = ld64(s);
      if ((uint32_t)(v >> 32) == (uint32_t)(h + 1ull)) {
        cell = (int)(uint32_t)v;
        st_coh(s, (h + (unsigned long long)q.cap) << 32);
        break;
      }
      if ((++spins & 15) == 0 &&
          (ld64(&e.ctl->active) == 0ull || get_err(e.ctl) || past_deadline(e.ctl)))
        break;
      if (spins < 64) __builtin_amdgcn_s_sleep(1);
      else __builtin_amdgcn_s_sleep(4);
    }
  }
  return bcast(cell, 0);
}

// Releases the band count a processed cell held.  One lane.
__device__ __forceinline__ void q_done(const Engine& e, int ring) {
  if (e.q.nb > 1) {
    order_release();
    atomic_add_relaxed(ctr(e.q.inflight, (uint32_t)ring), ~0ull);
  }
}

// ----------------------------------------------------------------------------
// heap schedule (one worker wave): the pending cell with the smallest
// (cell value, cell index) -- the heap order of the Heap-Cell Methods
// (Section 3.2.2) with the oracle's tie rule -- found through per-block minima
// ----------------------------------------------------------------------------

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned long long y = __shfl_xor(v, o, 64);
    v = y < v ? y : v;
  }
  return v;
}

// Key of cell c if it is pending and not running, else kKeyNone.
__device__ __forceinline__ unsigned long long pending_key(const Engine& e, int c) {
  if (c >= e.ncells) return kKeyNone;
  const uint32_t st = ld_coh(&e.st[c]);
  if (!(st & kPending) || (st & kRunning)) return kKeyNone;
  return ld_coh(&e.key[c]);
}

// Recomputes the minimum of block b (wave-cooperative).
__device__ __forceinline__ void heap_fix(const Engine& e, int b, int lane) {
  if (b < 0 || b >= ((e.ncells + 63) >> 6)) return;
  const unsigned long long m = wave_min_u64(pending_key(e, b * 64 + lane));
  if (lane == 0) st_coh(&e.hblk[b], m);
}

// The pending cell with the smallest (key, index), or -1 (wave-uniform).
// Blocks are scanned in index order, so among equal minima the lowest block
// -- which holds the lowest cell index with that key -- wins.
__device__ __forceinline__ int heap_pop(const Engine& e, int lane) {
  const int nblk = (e.ncells + 63) >> 6;
  unsigned long long best = kKeyNone;
  int bb = 0x7fffffff;
  for (int b = lane; b < nblk; b += 64) {
    const unsigned long long v = ld_coh(&e.hblk[b]);
    if (v < best) {
      best = v;
      bb = b;
    }
  }
  const unsigned long long m = wave_min_u64(best);
  if (m == kKeyNone) return -1;
  const int blk = __builtin_amdgcn_readfirstlane(wave::min_i(best == m ? bb : 0x7fffffff));
  const unsigned long long k = pending_key(e, blk * 64 + lane);
  const unsigned long long km = wave_min_u64(k);
  if (km == kKeyNone) return -1;  // not reached: the block minimum is kept current
  const unsigned long long at = ballot(k == km);
  return blk * 64 + __builtin_ctzll(at);
}

// Per-instance counts of cells waiting, queued or running (early
// completion): +1 when a cell of the instance becomes active, -1 when it
// goes idle; the wave whose decrement empties the count publishes the
// instance's completion to the host (its values were stored with
// device-scope accesses before every decrement of the chain).
// Active cells (waiting, queued or running).  A single problem keeps one
// count, ctl->active.  A batch keeps a count per problem (iact) and in
// ctl->active the number of problems with active cells: the per-visit
// updates spread over the problems' counters instead of meeting on one
// address, and ctl->active still reaches zero exactly when no cell is
// active.  A problem's count reaches zero once, when it is solved (a cell
// becomes active only through an active neighbour, and the preparation
// kernels have counted every initially active cell before the solver starts).
__device__ __forceinline__ void cell_active(const Engine& e, int g) {
  if (e.ninst > 1) atomic_add_relaxed(&e.iact[inst_index(e, g)], 1ull);
  else atomic_add_relaxed(&e.ctl->active, 1ull);
}
__device__ __forceinline__ void cell_idle(const Engine& e, int g) {
  if (e.ninst == 1) {
    atomic_add_relaxed(&e.ctl->active, ~0ull);
    return;
  }
  const int k = inst_index(e, g);
  if (atomic_add_relaxed(&e.iact[k], ~0ull) == 1ull) {
    if (e.idone) __hip_atomic_store(&e.idone[k], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    atomic_add_relaxed(&e.ctl->active, ~0ull);
  }
}

// Counts a cell removal against the visit guard (one lane).  A batch counts
// per problem (istat[4k], the problem's statistic too) against the problem's
// share of the guard: 64 J_k + 1024 by default, else the caller's limit
// scaled by J_k / J (at least 1).  A single problem counts in ctl->visits.
__device__ __forceinline__ void count_visit(const Engine& e, const Inst& I, int g) {
  if (e.ninst > 1) {
    const unsigned long long jk = (unsigned long long)I.kx * I.ky;
    unsigned long long lim = 64ull * jk + 1024ull;
    if (e.guard_given) {  // guard * jk / J without overflow (jk <= J < 2^31)
      const unsigned long long J = (unsigned long long)e.ncells, q = e.guard / J;
      lim = q > ~0ull / jk ? ~0ull : q * jk + (e.guard % J) * jk / J;
      if (lim < 1ull) lim = 1ull;
    }
    if (atomic_add_relaxed(e.istat + 4 * (size_t)inst_index(e, g), 1ull) >= lim)
      set_err(e.ctl, kErrGuard);
    return;
  }
  if (atomic_add_relaxed(&e.ctl->visits, 1ull) >= e.guard) set_err(e.ctl, kErrGuard);
}

// ----------------------------------------------------------------------------
// cell state transitions (one lane)
// ----------------------------------------------------------------------------

// A neighbour on side `sides` (bit mask, 0 for none) found that cell g must
// be processed (again), with preferred directions fl.  Enqueued when it is
// idle and its first processing is done; a running cell takes the request
// itself when it finishes, and a cell still waiting for its first processing
// reads the new values when it starts.
// Under the heap schedule a queued cell is only marked pending: the single
// worker finds it by its cell value (heap_pop).
template <bool RINGS = true>
__device__ void requeue(const Engine& e, int g, uint32_t fl, uint32_t sides, double key) {
  order_release();
  const uint32_t old =
      __hip_atomic_fetch_or(&e.st[g], kPending | (fl << kFlagShift) | (sides << kSideShift),
                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!(old & (kPending | kRunning)) && (old & kDone1)) {
    cell_active(e, g);
    if (e.ready_at) e.ready_at[g] = wall_clock64();
    if (!e.heap) q_push<RINGS>(e, (uint32_t)g, key);
  }
}

// The last earlier neighbour of cell g finished its first processing: g is
// enqueued (only this path enqueues a cell before its first processing).
template <bool RINGS = true>
__device__ void release_first(const Engine& e, int g) {
  order_release();
  __hip_atomic_fetch_or(&e.st[g], kPending, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (e.ready_at) e.ready_at[g] = wall_clock64();
  q_push<RINGS>(e, (uint32_t)g, 0.0);
}

// Takes a popped (or re-requested) cell: state -> running, keeping kDone1.
// Returns the previous state word.
__device__ uint32_t claim(const Engine& e, int g) {
  uint32_t old = ld_coh(&e.st[g]);
  for (;;) {
    const uint32_t want = (old & kDone1) | kRunning;
    if (__hip_atomic_compare_exchange_strong(&e.st[g], &old, want, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      break;
  }
  return old;
}

// ----------------------------------------------------------------------------
// sweeps
// ----------------------------------------------------------------------------

// One Gauss-Seidel sweep in direction dir (0 SW, 1 NW, 2 NE, 3 SE: x and y
// ascending for SW, x ascending / y descending for NW, ...) over the w x hgt
// tile in LDS (pitch P, halo at row/column 0 and w+1/hgt+1; the halo's h/F
// is +inf, see halo_to_masks).  Returns (wave-uniform) bit 0: some node
// decreased;
// bit 1 (bit 2): some node that decreased is now below its upwind neighbour
// in x (in y) inside the tile.  Without bits 1 and 2 the tile is converged:
// every node was
// evaluated with its upwind neighbours' final values, and a node can only be
// lowered further through a downwind neighbour that fell below it during the
// sweep (a neighbour that stays at or above it cannot lower it, by the
// causality of the update).  DIRECTIONAL uses only the two upwind neighbours
// of the sweep (the sweep-directional update of FMSM) instead of the
// quadrant shortcut.
//
// At step d lane l updates node (i, j) with i = column l in sweep order and j
// = row t = d - l in sweep order.  The upwind x-neighbour is lane l-1's result
// of step d-1 (for lane 0 the halo value, supplied as the DPP's out-of-range
// operand); the upwind y-neighbour is the lane's own previous result, which
// before the lane's first row holds the halo value below it.  The step is
// branch-free, and with no select: a lane whose row lies outside the tile
// (clamped to a halo row), or which lies past the tile's width (on the halo
// column beside the tile), updates a halo node, whose h/F of +inf makes the
// update "no update", so it stores back the value it read and carries that
// halo value as its upwind value, as the lane's first row needs.  The old
// values a step needs are read one step ahead (none is a location the
// current step writes); the node's own old value is the north value read for
// the step before.  min is v_min_f64, which also maps the NaN that a = b =
// +inf (or an infinite h/F) produces to "no update", as the oracle's explicit
// test does.
// STATS: also the lane's largest decrease (+inf for a node that left +inf)
// and number of decreased nodes, into *mx and *cnt.  FAITHFUL: the update's
// root within one unit in the last place (local_update).
// The three result bits are kept as wave masks (lanes that decreased, and
// that did so below an upwind neighbour), one scalar AND / OR per term and
// step; lane 0's x-neighbour is the fixed halo, so its bit is dropped at the
// end.
template <typename T, int P, bool DIRECTIONAL, bool STATS, int dir, bool FAITHFUL = false>
__device__ __forceinline__ uint32_t sweep_tile_dir(T* tu, const T* td, int w, int hgt, int lane,
                                                   double* mx, int* cnt) {
  lane = opaque_lane(lane);
  double smx = 0.0;
  int scnt = 0;
  const int sx = (dir == 0 || dir == 1) ? 1 : -1;
  const int sy = (dir == 0 || dir == 3) ? 1 : -1;
  const int rowstep = sy * P;
  const bool col_ok = lane < w;
  // lanes past the tile's width walk the halo column on the sweep's far side
  const int i = col_ok ? (sx > 0 ? lane : w - 1 - lane) : (sx > 0 ? w : -1);
  const int j0 = sy > 0 ? 0 : hgt - 1;
  const int nsteps = __builtin_amdgcn_readfirstlane(w + hgt - 1);  // the same on every lane
  // LDS index of the lane's node at sweep-order row t, clamped to the halo rows
  auto idx_t = [&](int t) {
    const int tc = t < -1 ? -1 : (t > hgt ? hgt : t);
    return (j0 + sy * tc + 1) * P + i + 1;
  };
  int c = idx_t(-lane), c1 = idx_t(1 - lane);  // the lane's positions at steps 0 and 1
  T prev = tu[idx_t(-1)];
  unsigned long long m_dec = 0ull, m_bx = 0ull, m_by = 0ull;
  const unsigned long long m_col = ballot(col_ok);
  // One step at d: the node's old value uo and its north value nv were read
  // before; the values of the next step are read into the *n references.
  // The lane's row index moves by one row while t + 1 lies in [0, hgt].  The
  // value read as the next step's north value is the one at the lane's
  // position two steps on (the north neighbour wherever the lane has a node),
  // so that it is also that step's own old value where the row is clamped.
  auto step = [&](int d, const T& ev, const T& uo, const T& nv, const T& dl, const T& hw,
                  T& evn, T& nvn, T& dln, T& hwn) {
    const int t = d - lane;
    const bool valid = col_ok && (unsigned)t < (unsigned)hgt;
    const int c2 = c1 + ((unsigned)(t + 2) <= (unsigned)hgt ? rowstep : 0);
    evn = tu[c1 + sx];
    nvn = tu[c2];
    dln = td[c1];
    hwn = tu[c1 - sx];
    const T wv = shr1_or(prev, hw);
    const T a = DIRECTIONAL ? wv : vmin(wv, ev);
    const T b = DIRECTIONAL ? prev : vmin(prev, nv);
    const T U = local_update<FAITHFUL>(a, b, dl);
    const T r = vmin(uo, U);
    const bool dec = valid && (r < uo);
    // ballot(dec), as three compare masks (no detour through a register)
    const unsigned long long md = ballot(r < uo) & ballot((unsigned)t < (unsigned)hgt) & m_col;
    m_dec |= md;
    m_bx |= md & ballot(r < wv);
    m_by |= md & ballot(r < prev) & ballot(t > 0);
    if constexpr (STATS) {
      const double chg = (double)uo - (double)r;  // +inf when uo is +inf
      smx = dec && chg > smx ? chg : smx;
      scnt += dec ? 1 : 0;
    }
    tu[c] = r;
    prev = r;
    c = c1;
    c1 = c2;
  };
  // two steps per iteration (the step count is wave-uniform): the values
  // read one step ahead alternate between two register sets
  T evA = tu[c + sx], nvA = tu[c1], uoA = tu[c], dlA = td[c], hwA = tu[c - sx];
  T evB, nvB, dlB, hwB;
  int d = 0;
  for (; d + 1 < nsteps; d += 2) {
    step(d, evA, uoA, nvA, dlA, hwA, evB, nvB, dlB, hwB);
    step(d + 1, evB, nvA, nvB, dlB, hwB, evA, uoA, dlA, hwA);
    // the next north value was read into uoA; the old value is nvB
    const T nn = uoA;
    uoA = nvB;
    nvA = nn;
  }
  if (d < nsteps) step(d, evA, uoA, nvA, dlA, hwA, evB, nvB, dlB, hwB);
  if constexpr (STATS) {
    *mx = smx;
    *cnt = scnt;
  }
  return (m_dec ? 1u : 0u) | ((m_bx & ~1ull) ? 2u : 0u) | (m_by ? 4u : 0u);
}

// The sweep with its direction fixed at compile time (the neighbour offsets
// become immediates of the LDS accesses).
template <typename T, int P, bool DIRECTIONAL, bool STATS = false, bool FAITHFUL = false>
__device__ uint32_t sweep_tile(T* tu, const T* td, int w, int hgt, int dir, int lane,
                               double* mx = nullptr, int* cnt = nullptr) {
  switch (dir) {
    case 0: return sweep_tile_dir<T, P, DIRECTIONAL, STATS, 0, FAITHFUL>(tu, td, w, hgt, lane, mx, cnt);
    case 1: return sweep_tile_dir<T, P, DIRECTIONAL, STATS, 1, FAITHFUL>(tu, td, w, hgt, lane, mx, cnt);
    case 2: return sweep_tile_dir<T, P, DIRECTIONAL, STATS, 2, FAITHFUL>(tu, td, w, hgt, lane, mx, cnt);
    default: return sweep_tile_dir<T, P, DIRECTIONAL, STATS, 3, FAITHFUL>(tu, td, w, hgt, lane, mx, cnt);
  }
}

// After a tile load: records per side which outside nodes are accessible
// (finite h/F) as a mask along the side (bit k: row k for W/E, column k for
// S/N) in hacc[0..3] (W, E, S, N; when hacc is given), and sets the halo's
// h/F, corners included, to +inf, which the sweep relies on (sweep_tile_dir).
// One wave, after every part of the load has landed.
template <typename T, int P>
__device__ void halo_to_masks(T* td, int w, int hgt, int lane, unsigned long long* hacc) {
  lane = opaque_lane(lane);
  const T INF = inf_v<T>();
  const bool rv = lane < hgt, cv = lane < w;
  const int iw = (lane + 1) * P, ie = iw + w + 1, is = lane + 1, in = (hgt + 1) * P + lane + 1;
  const T dW = rv ? td[iw] : INF, dE = rv ? td[ie] : INF;
  const T dS = cv ? td[is] : INF, dN = cv ? td[in] : INF;
  const unsigned long long mW = ballot(dW != INF), mE = ballot(dE != INF);
  const unsigned long long mS = ballot(dS != INF), mN = ballot(dN != INF);
  if (rv) {
    td[iw] = INF;
    td[ie] = INF;
  }
  if (cv) {
    td[is] = INF;
    td[in] = INF;
  }
  if (lane < 4) td[lane == 0 ? 0 : lane == 1 ? w + 1 : lane == 2 ? (hgt + 1) * P : (hgt + 1) * P + w + 1] = INF;
  if (hacc && lane == 0) {
    hacc[0] = mW;
    hacc[1] = mE;
    hacc[2] = mS;
    hacc[3] = mN;
  }
}

// Convergence test of the tile against its halo: true when no node would
// decrease, T(V) >= V everywhere.  A Gauss-Seidel sweep that changes nothing
// is exactly this test, but the test has no dependency chain between nodes:
// each lane walks its column.
template <typename T, int P>
__device__ bool tile_converged(const T* tu, const T* td, int w, int hgt, int lane) {
  lane = opaque_lane(lane);
  bool bad = false;
  if (lane < w) {
#pragma unroll 4
    for (int j = 0; j < hgt; ++j) {
      const int k = (j + 1) * P + lane + 1;
      const T a = vmin(tu[k - 1], tu[k + 1]);
      const T b = vmin(tu[k - P], tu[k + P]);
      const T U = local_update(a, b, td[k]);
      bad |= U < tu[k];
    }
  }
  return ballot(bad) == 0ull;
}

// FMSM sweep directions (bit d = direction d: 0 SW, 1 NW, 2 NE, 3 SE) from
// the sides (bit 0 W, 1 E, 2 S, 3 N) whose neighbour was accepted earlier,
// following the figure on coarse sweep choice: sweeps start from the corners
// formed by an earlier vertical and an earlier horizontal side; with earlier
// sides on one axis only, both corners of each such side.
__device__ __forceinline__ uint32_t fmsm_dirs(uint32_t sides) {
  const bool W = sides & 1u, E = sides & 2u, S = sides & 4u, N = sides & 8u;
  uint32_t d = 0;
  if ((W || E) && (S || N)) {
    if (S && W) d |= 1u;
    if (N && W) d |= 2u;
    if (N && E) d |= 4u;
    if (S && E) d |= 8u;
  } else {
    if (W) d |= 1u | 2u;
    if (E) d |= 4u | 8u;
    if (S) d |= 1u | 8u;
    if (N) d |= 2u | 4u;
  }
  return d;
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

// ----------------------------------------------------------------------------
// tiles in LDS
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
// delta into LDS; outside the grid: +inf.  Rows go straight from memory into
// LDS (global_load_lds: each active lane moves 16 bytes of the row), so the
// loads of every row of the tile are in flight together without holding any
// data in registers (the cell solver uses load_tile_v below, through
// registers, which is faster where the registers suffice); u is read with the
// coherent policy (sc1) because neighbouring cells write it concurrently.  The west and east halo columns
// (one element per row) go through registers.  One wait at the end.
// fresh: the cell has never been processed and holds no exit node, so its
// interior values are all +inf and only delta and the halo are read.
// part / nparts: this wave loads rows r with (r + 1) mod nparts == part and,
// as part 0, the west and east halo columns (several waves of a workgroup
// share one tile load).
template <typename T, int P>
__device__ void load_tile(T* tu, T* td, const Inst& I, const CellBox& B, int lane,
                          bool with_interior, bool fresh = false, int part = 0, int nparts = 1) {
  lane = opaque_lane(lane);
  using lds_ptr = __attribute__((address_space(3))) void*;
  constexpr int kCohPolicy = 16;             // sc1
  // the cell box and grid are the same on every lane: scalar loop control
  // and row addresses
  auto uni_ptr = [](const void* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<const char*>((uint64_t)hi << 32 | lo);
  };
  const char* ub = uni_ptr(I.u);
  const char* db = uni_ptr(I.delta);
  const T INF = inf_v<T>();
  const int nx = __builtin_amdgcn_readfirstlane(I.nx), ny = __builtin_amdgcn_readfirstlane(I.ny);
  const int bw = __builtin_amdgcn_readfirstlane(B.w), bh = __builtin_amdgcn_readfirstlane(B.hgt);
  const int bx0 = __builtin_amdgcn_readfirstlane(B.x0), by0 = __builtin_amdgcn_readfirstlane(B.y0);
  const int rowbytes = bw * (int)sizeof(T);
  const int n16 = rowbytes >> 4;           // full 16-byte pieces of a row
  const int tail_dw = (rowbytes & 15) >> 2;  // remaining dwords
  for (int r = -1; r <= bh; ++r) {
    const bool halo_row = r < 0 || r == bh;
    if (!with_interior && !halo_row) {
      r = bh - 1;  // skip to the north halo row
      continue;
    }
    if (nparts > 1 && (r + 1) % nparts != part) continue;
    const int j = by0 + r;
    T* lu = tu + (r + 1) * P + 1;
    T* ld = td + (r + 1) * P + 1;
    if (j < 0 || j >= ny) {
      if (lane < bw) {
        lu[lane] = INF;
        ld[lane] = INF;
      }
      continue;
    }
    const bool skip_u = fresh && !halo_row;
    const size_t row = ((size_t)j * nx + bx0) * sizeof(T);
    // 16 bytes per lane for the bulk of the row, then single dwords for the
    // ragged end (rows are at most 512 bytes: one instruction each)
    if (lane < n16) {
      if (!skip_u)
        __builtin_amdgcn_global_load_lds(ub + row + 16 * (size_t)lane, (lds_ptr)lu, 16, 0, kCohPolicy);
      __builtin_amdgcn_global_load_lds(db + row + 16 * (size_t)lane, (lds_ptr)ld, 16, 0, 0);
    }
    if (tail_dw) {
      if (lane < tail_dw) {
        const size_t at = row + 16 * (size_t)n16 + 4 * (size_t)lane;
        if (!skip_u)
          __builtin_amdgcn_global_load_lds(ub + at, (lds_ptr)((char*)lu + 16 * n16), 4, 0, kCohPolicy);
        __builtin_amdgcn_global_load_lds(db + at, (lds_ptr)((char*)ld + 16 * n16), 4, 0, 0);
      }
    }
    if (skip_u && lane < bw) lu[lane] = INF;
  }
  if (part == 0) {
    const gptr<const T> u = to_global(static_cast<const T*>(I.u));
    const gptr<const T> dl = to_global(static_cast<const T*>(I.delta));
    const int jr = B.y0 + (lane < B.hgt ? lane : 0);
    const size_t rowi = (size_t)jr * nx;
    const int iw = B.x0 > 0 ? B.x0 - 1 : 0;
    const int ie = B.x1 < nx ? B.x1 : nx - 1;
    const T vw = ld_coh(u + rowi + iw), dw = dl[rowi + iw];
    const T ve = ld_coh(u + rowi + ie), de = dl[rowi + ie];
    if (lane < B.hgt) {
      tu[(lane + 1) * P] = B.x0 > 0 ? vw : INF;
      td[(lane + 1) * P] = B.x0 > 0 ? dw : INF;
      tu[(lane + 1) * P + B.w + 1] = B.x1 < nx ? ve : INF;
      td[(lane + 1) * P + B.w + 1] = B.x1 < nx ? de : INF;
    }
  }
  // the row transfers write LDS asynchronously: wait for all of them
  __builtin_amdgcn_s_waitcnt(0);
}

// The same tile load through registers: the lanes move 16-byte pieces of
// the rows with buffer loads, a fixed number of lanes per row (the row's
// pieces, rounded up to a power of two) and several rows per instruction,
// all of a lane's pieces in flight at once (u with the coherent sc1 policy;
// loads past the array's end return zeros and are never used), then write
// the elements that belong to the row into LDS.  Rows as in load_tile: this
// wave loads rows ri = part, part + NW, ... of the rows the call loads (at
// most ROWS).  Arrays of 4 GiB or more, and tiles with more than nine
// instructions' worth of rows per wave (64-node cells loaded by one wave),
// take load_tile.
template <typename T, int P, int NW, int ROWS = P>
__device__ void load_tile_v(T* tu, T* td, const Inst& I, const CellBox& B, int lane,
                            bool with_interior, bool fresh, int part) {
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  constexpr int kEl = 16 / (int)sizeof(T);  // elements per piece
  constexpr int kPieces = (P - 2 + kEl - 1) / kEl;
  constexpr int kLanesPerRow = kPieces <= 4 ? 4 : kPieces <= 8 ? 8 : kPieces <= 16 ? 16 : 32;
  constexpr int kRowsPerInstr = 64 / kLanesPerRow;
  constexpr int kRowsPerWave = (ROWS + NW - 1) / NW;
  constexpr int kMax = (kRowsPerWave + kRowsPerInstr - 1) / kRowsPerInstr;
  constexpr int kCohPolicy = 16;  // sc1
  if constexpr (kMax > 9) {  // more rows per wave than registers to hold them
    load_tile<T, P>(tu, td, I, B, lane, with_interior, fresh, part, NW);
    return;
  }
  if ((size_t)I.nx * I.ny * sizeof(T) >= (1ull << 32)) {
    load_tile<T, P>(tu, td, I, B, lane, with_interior, fresh, part, NW);
    return;
  }
  lane = opaque_lane(lane);
  const T INF = inf_v<T>();
  const int nx = __builtin_amdgcn_readfirstlane(I.nx), ny = __builtin_amdgcn_readfirstlane(I.ny);
  const int bw = __builtin_amdgcn_readfirstlane(B.w), bh = __builtin_amdgcn_readfirstlane(B.hgt);
  const int bx0 = __builtin_amdgcn_readfirstlane(B.x0), by0 = __builtin_amdgcn_readfirstlane(B.y0);
  const int nrow_all = with_interior ? bh + 2 : 2;
  const uint32_t bytes = (uint32_t)((size_t)nx * ny * sizeof(T));
  const __amdgpu_buffer_rsrc_t ru =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(I.u), 0, bytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t rd =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(I.delta), 0, bytes, 0x00020000);
  const int col = (lane % kLanesPerRow) * kEl;  // first element of the lane's piece
  const int sub = lane / kLanesPerRow;          // row within an instruction's rows
  v4u pu[kMax], pd[kMax];
#pragma unroll
  for (int k = 0; k < kMax; ++k) {
    const int ri = part + NW * (k * kRowsPerInstr + sub);
    const int r = with_interior ? ri - 1 : (ri == 0 ? -1 : bh);
    const int j = by0 + r;
    const bool live = ri < nrow_all && col < bw && j >= 0 && j < ny;
    const bool want_u = live && (!fresh || r < 0 || r == bh);
    const uint32_t off = live ? (uint32_t)(j * nx + bx0 + col) * (uint32_t)sizeof(T) : 0u;
    pu[k] = want_u ? __builtin_amdgcn_raw_buffer_load_b128(ru, off, 0, kCohPolicy) : v4u{0u, 0u, 0u, 0u};
    pd[k] = live ? __builtin_amdgcn_raw_buffer_load_b128(rd, off, 0, 0) : v4u{0u, 0u, 0u, 0u};
  }
#pragma unroll
  for (int k = 0; k < kMax; ++k) {
    const int ri = part + NW * (k * kRowsPerInstr + sub);
    const int r = with_interior ? ri - 1 : (ri == 0 ? -1 : bh);
    const int j = by0 + r;
    if (ri >= nrow_all || col >= bw) continue;
    const bool in_grid = j >= 0 && j < ny;
    const bool want_u = in_grid && (!fresh || r < 0 || r == bh);
    T eu[kEl], ed[kEl];
    __builtin_memcpy(eu, &pu[k], 16);
    __builtin_memcpy(ed, &pd[k], 16);
    T* lu = tu + (r + 1) * P + 1 + col;
    T* ld = td + (r + 1) * P + 1 + col;
#pragma unroll
    for (int m = 0; m < kEl; ++m) {
      if (col + m < bw) {
        lu[m] = want_u ? eu[m] : INF;
        ld[m] = in_grid ? ed[m] : INF;
      }
    }
  }
  if (part == 0) {
    const gptr<const T> u = to_global(static_cast<const T*>(I.u));
    const gptr<const T> dl = to_global(static_cast<const T*>(I.delta));
    const int jr = B.y0 + (lane < B.hgt ? lane : 0);
    const size_t rowi = (size_t)jr * nx;
    const int iw = B.x0 > 0 ? B.x0 - 1 : 0;
    const int ie = B.x1 < nx ? B.x1 : nx - 1;
    const T vw = ld_coh(u + rowi + iw), dw = dl[rowi + iw];
    const T ve = ld_coh(u + rowi + ie), de = dl[rowi + ie];
    if (lane < B.hgt) {
      tu[(lane + 1) * P] = B.x0 > 0 ? vw : INF;
      td[(lane + 1) * P] = B.x0 > 0 ? dw : INF;
      tu[(lane + 1) * P + B.w + 1] = B.x1 < nx ? ve : INF;
      td[(lane + 1) * P + B.w + 1] = B.x1 < nx ? de : INF;
    }
  }
}

// Writes the whole tile back to u.
template <typename T, int P>
__device__ void store_tile(const T* tu, const Inst& I, const CellBox& B, int lane, int part = 0,
                           int nparts = 1) {
  lane = opaque_lane(lane);
  T* u = static_cast<T*>(I.u);
  if (lane < B.w)
    for (int r = part; r < B.hgt; r += nparts)
      st_coh(u + (size_t)(B.y0 + r) * I.nx + B.x0 + lane, tu[(r + 1) * P + lane + 1]);
}

// Work that the helper waves of a multi-wave workgroup share with wave 0:
// op 0 = leave, 1 = load cell g's tile (flags bit 0 with_interior, bit 1
// fresh), 2 = store cell g's tile.  Wave 0 writes the job, then every wave
// passes barrier A, does its share, waits for its own transfers and passes
// barrier B; each job is exactly one A-B pair for every wave (leave: A only).
struct TileJob {
  int op, g, flags;
};

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
  const double* Fd = static_cast<const double*>(I.F);
  double sum = 0.0;
  int cnt = 0;
  for (int m = 0; m < np; ++m) {
    const int ii = side <= 1 ? p[m] : other;
    const int jj = side <= 1 ? other : p[m];
    if (ii < 0 || jj < 0 || ii >= I.nx || jj >= I.ny) continue;
    const size_t k = (size_t)jj * I.nx + ii;
    if (I.mask && !I.mask[k]) continue;
    sum += I.qdense ? Fd[k] : (double)F[k];
    cnt++;
  }
  return cnt ? sum / cnt : 0.0;
}

// wave-wide max of x (never NaN) with the lowest lane attaining it
// (x = -inf on every lane: none, *arg = -1)
__device__ __forceinline__ double wave_max(double x, int* arg) {
  const double m = wave::max_d(x);
  const unsigned long long at = ballot(x == m && m > -__builtin_huge_val());
  *arg = at ? __builtin_ctzll(at) : -1;
  return m;
}

// Monotonicity of the finite values v of the lanes in `fin`, in ascending
// lane order: bit 0 non-decreasing, bit 1 non-increasing (wave-uniform).
template <typename T>
__device__ uint32_t line_monotone(T v, bool fin, int lane) {
  const unsigned long long m = ballot(fin);
  const unsigned long long below = m & ((1ull << lane) - 1ull);
  const int pred = below ? 63 - __builtin_clzll(below) : lane;
  const T pv = __shfl(v, pred, 64);
  const bool has = fin && below;
  const bool up_bad = has && pv > v;
  const bool down_bad = has && pv < v;
  return (ballot(up_bad) ? 0u : 1u) | (ballot(down_bad) ? 0u : 2u);
}

// After processing: writes the boundary nodes that decreased since they were
// last published, re-queues neighbours by the add criterion of Algorithm
// generic_LC_cells (FHCM narrows the raised directions by the monotonicity
// check of Algorithm FHCM), and lowers their cell values (eq. cell_value).
template <typename T, int P, int M, bool RINGS>
__device__ void publish(const Engine& e, const Inst& I, const CellBox& B, int g, T* tu,
                        const T* td, const unsigned long long* hacc, T pub[4], bool first, int lane) {
  lane = opaque_lane(lane);
  const T INF = inf_v<T>();
  T* u = static_cast<T*>(I.u);
  // per side: add criterion met somewhere, max finite value and its lane,
  // monotonicity; lane `side` keeps side's results
  bool my_crit = false;
  double my_kv = -__builtin_huge_val();
  int my_karg = -1;
  uint32_t my_mono = 3u;
#pragma nounroll
  for (int side = 0; side < 4; ++side) {
    // side 0 W: column 0, 1 E: column w-1 (lane = row); 2 S: row 0, 3 N: row
    // hgt-1 (lane = column)
    const bool vert = side <= 1;
    const int len = vert ? B.hgt : B.w;
    const bool ok = lane < len;
    const int step = vert ? P : 1;      // LDS stride along the side
    const int out = side == 0 ? -1 : side == 1 ? 1 : side == 2 ? -P : P;
    const int base = side == 0 ? P + 1 : side == 1 ? P + B.w : side == 2 ? P + 1 : B.hgt * P + 1;
    const int idx_in = ok ? base + lane * step : P + 1;
    const int idx_out = ok ? idx_in + out : P + 1;
    const T ps = side == 0 ? pub[0] : side == 1 ? pub[1] : side == 2 ? pub[2] : pub[3];
    const T v = tu[idx_in];
    bool c = false;
    double vmax = -__builtin_huge_val();
    if (ok) {
      const bool is_src = td[idx_in] == INF && v != INF;
      const bool changed = v < ps || (first && is_src);
      if (v < ps) {
        const int ii = vert ? (side == 0 ? B.x0 : B.x1 - 1) : B.x0 + lane;
        const int jj = vert ? B.y0 + lane : (side == 2 ? B.y0 : B.y1 - 1);
        st_coh(u + (size_t)jj * I.nx + ii, v);
      }
      c = changed && ((hacc[side] >> lane) & 1ull) && v < tu[idx_out];
      if (v != INF) vmax = (double)v;
    }
    const T np = ok ? v : ps;
    if (side == 0) pub[0] = np;
    else if (side == 1) pub[1] = np;
    else if (side == 2) pub[2] = np;
    else pub[3] = np;
    const bool cr = ballot(c) != 0ull;
    // the boundary maximum only feeds the neighbour's key (schedules other
    // than the dependency order)
    int ka = -1;
    const double kvv = e.dag ? -__builtin_huge_val() : wave_max(vmax, &ka);
    const uint32_t mo = M == kFhcm ? line_monotone(v, ok && v != INF, lane) : 3u;
    if (lane == side) {
      my_crit = cr;
      my_kv = kvv;
      my_karg = ka;
      my_mono = mo;
    }
  }
  // make the boundary values visible before any neighbour is signalled
  order_release();
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
      double key = __builtin_huge_val();
      if (!e.dag && my_karg >= 0) {
        const int along = side == 0 ? B.x0 : side == 1 ? B.x1 - 1 : side == 2 ? B.y0 : B.y1 - 1;
        const int other = side <= 1 ? B.y0 + my_karg : B.x0 + my_karg;
        const double fy = speed_at<T>(I, side, along, other, wk);
        if (fy > 0.0) {
          key = my_kv + (0.5 * (1 + wk) * I.h) / fy;
          const unsigned long long old = __hip_atomic_fetch_min(
              &e.key[nb], key_bits(key), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const double okey = key_value(old);
          if (okey < key) key = okey;
        }
      }
      if (my_crit) {
        const int recv = side ^ 1;  // the receiving cell sees us on the opposite side
        uint32_t dirs = side_dirs(recv);
        if (M == kFhcm) {
          // line order N->S for W/E lines (descending lanes), W->E for S/N lines
          const uint32_t m = my_mono;
          const bool nondec = side <= 1 ? (m & 2u) : (m & 1u);
          const bool noninc = side <= 1 ? (m & 1u) : (m & 2u);
          atomic_add_relaxed(&e.ctl->mon_checks, 1ull);
          if (nondec || noninc) atomic_add_relaxed(&e.ctl->mon_ok, 1ull);
          if (nondec != noninc) {
            // receiver's west side: NW / SW; east: NE / SE; north: NW / NE;
            // south: SW / SE (first = line non-decreasing)
            const uint32_t a = recv == 0 ? 0x2u : recv == 1 ? 0x4u : recv == 3 ? 0x2u : 0x1u;
            const uint32_t b = recv == 0 ? 0x1u : recv == 1 ? 0x8u : recv == 3 ? 0x4u : 0x8u;
            dirs = nondec ? a : b;
          }
        }
        requeue<RINGS>(e, nb, dirs, 1u << recv, key);
      }
    }
  }
}

// ----------------------------------------------------------------------------
// persistent solver kernel
// ----------------------------------------------------------------------------

// First processing of cell g done: a later neighbour starts once all its
// earlier neighbours are done.  One lane.
// Side `side` (0..3) of cell g: its later neighbour there loses one
// dependency and starts when none is left.  Lanes 0..3 call it for one side
// each, so the four dependency counts and queue pushes (chains of
// device-scope atomics) proceed at once.
template <bool RINGS>
__device__ void release_later(const Engine& e, int g, const Inst& I, const CellBox& B,
                              uint32_t ordb, int side) {
  int nb = -1;
  if (side == 0 && B.cx > 0) nb = g - 1;
  if (side == 1 && B.cx + 1 < I.kx) nb = g + 1;
  if (side == 2 && B.cy > 0) nb = g - I.kx;
  if (side == 3 && B.cy + 1 < I.ky) nb = g + I.kx;
  if (nb < 0 || (ordb & (1u << side))) return;  // none, or earlier
  if (e.ord[nb] & kOrdEmpty) return;
  if (atomic_add_relaxed(&e.deps[nb], -1) == 1) release_first<RINGS>(e, nb);
}

// NW waves per workgroup: wave 0 runs the worker; with NW > 1 (single
// problems, where compute units are plentiful) waves 1..NW-1 only share the
// tile loads and stores, which one wave issues at one row transfer per
// ~70-90 cycles.
constexpr int kSolveWaves1 = 4;  // waves per worker for single problems

// LDS of a tile with pitch P: one guard row, the (P x P) tile with its halo
// and 65 guard elements.  The sweep reads the next step's operands one step
// ahead, and on its last steps that read reaches one row beyond the far halo
// row (south: row -1, down to -P; north: up to P*P + 64 for 64-node cells);
// the guards keep those reads, whose values are discarded, inside the array.
template <int P>
struct TileLds {
  static constexpr int kBefore = P;
  static constexpr int kSize = P + P * P + 64 + 1;
};

// HEAP: the heap schedule's single worker (a kernel of its own, so that the
// other schedules carry none of its code).
template <typename T, int S, int M, int NW, bool HEAP = false>
__global__ __launch_bounds__(64 * NW) void k_solve(Engine e) {
  constexpr int P = S + 2;
  __shared__ T tu_mem[TileLds<P>::kSize];
  T* const tu = tu_mem + TileLds<P>::kBefore;  // the tile with its halo
  __shared__ T td[P * P];
  __shared__ TileJob job;
  __shared__ unsigned long long hacc[4];  // accessible outside nodes per side
  const int lane = threadIdx.x & 63;
  if constexpr (NW > 1) {
    if (threadIdx.x >= 64) {  // helper wave
      const int part = threadIdx.x >> 6;
      for (;;) {
        __syncthreads();  // A
        const int op = __builtin_amdgcn_readfirstlane(job.op);
        const int g = __builtin_amdgcn_readfirstlane(job.g);
        const int flags = __builtin_amdgcn_readfirstlane(job.flags);
        if (op == 0) return;
        const Inst I = inst_of(e, g);
        const CellBox B = cell_box(I, g - I.cell0);
        if (op == 1) {
          load_tile_v<T, P, NW>(tu, td, I, B, lane, (flags & 1) != 0, (flags & 2) != 0, part);
        } else {
          store_tile<T, P>(tu, I, B, lane, part, NW);
          __builtin_amdgcn_s_waitcnt(0);
        }
        __syncthreads();  // B
      }
    }
  }
  auto tile_load = [&](const Inst& I, const CellBox& B, int g, bool with_interior, bool fresh) {
    if constexpr (NW == 1) {
      load_tile_v<T, P, 1>(tu, td, I, B, lane, with_interior, fresh, 0);
    } else {
      if (lane == 0) job = TileJob{1, g, (with_interior ? 1 : 0) | (fresh ? 2 : 0)};
      __syncthreads();  // A
      load_tile_v<T, P, NW>(tu, td, I, B, lane, with_interior, fresh, 0);
      __syncthreads();  // B: every part has landed
    }
    halo_to_masks<T, P>(td, B.w, B.hgt, lane, hacc);
  };
  auto tile_store = [&](const Inst& I, const CellBox& B, int g) {
    if constexpr (NW == 1) {
      store_tile<T, P>(tu, I, B, lane);
    } else {
      if (lane == 0) job = TileJob{2, g, 0};
      __syncthreads();  // A
      store_tile<T, P>(tu, I, B, lane, 0, NW);
      __syncthreads();  // B: the helpers' stores have completed
    }
  };
  Ctl* ctl = e.ctl;
  if (!get_err(ctl)) {
  int backoff = 0;
  unsigned long long t0 = kProfiling && e.profile ? wall_clock64() : 0ull;
  unsigned long long ph[kPhases] = {0, 0, 0, 0, 0, 0};
  unsigned long long nsweeps = 0, nchecks = 0;  // this wave's totals
  if constexpr (HEAP)  // the only worker: block minima of the cells queued so far
    for (int b = 0; b < ((e.ncells + 63) >> 6); ++b) heap_fix(e, b, lane);
  // under per-problem groups a wave looks at the group of its own index first;
  // a FIFO wave waits on the ring of its own index
  const uint32_t home = e.q.ng > 1                ? blockIdx.x % e.q.ng
                        : NW == 1 && e.q.nb == 1   ? blockIdx.x & (e.q.nring - 1u)
                                                   : 0u;
  for (;;) {
    int ring = 0;
    const int g = HEAP            ? heap_pop(e, lane)
                  : e.q.nb == 1   ? q_pop_ticket<(NW == 1)>(e, lane, home)
                  : e.q.ng > 1    ? q_pop_groups(e, lane, home, &ring)
                                  : q_pop(e, lane, &ring);
    if (g < 0) {
      const bool stop = HEAP || e.q.nb == 1 || ld64(&ctl->active) == 0ull || get_err(ctl) ||
                        past_deadline(ctl);
      if (stop) break;
      if (backoff < 8) ++backoff;
      for (int z = 0; z < backoff; ++z) __builtin_amdgcn_s_sleep(2);
      tick(e, ph, kPhIdle, &t0);
      continue;
    }
    backoff = 0;
    tick(e, ph, kPhIdle, &t0);  // waiting for a cell, the pop included
    unsigned long long tr[5] = {0, 0, 0, 0, 0};
    const unsigned long long sw0 = nsweeps, ch0 = nchecks;
    if (e.trace) tr[0] = wall_clock64();
    const Inst I = inst_of(e, g);  // by value: fields stay in registers
    const CellBox B = cell_box(I, g - I.cell0);
    uint32_t fl = 0, ordb = 0, sides = 0;
    int first = 0, done1 = 0;
    uint32_t run_state = kRunning;  // the state word written by claim (lane 0)
    // the claim's bookkeeping is spread over lanes 1-3 and issued before the
    // claim itself, so the device-scope round trips overlap
    if (lane == 1) first = atomic_add_relaxed(&e.visits[g], 1u) == 0u ? 1 : 0;
    if (lane == 2) count_visit(e, I, g);
    if (lane == 3 && e.dag) ordb = e.ord[g];
    if (lane == 0) {
      const uint32_t old = claim(e, g);
      run_state = (old & kDone1) | kRunning;
      fl = (old >> kFlagShift) & 0xFu;
      sides = (old >> kSideShift) & 0xFu;
      done1 = (old & kDone1) != 0u;
    }
    fl = (uint32_t)bcast((int)fl, 0);
    sides = (uint32_t)bcast((int)sides, 0);
    ordb = (uint32_t)bcast((int)ordb, 3);
    done1 = bcast(done1, 0);
    bool is_first = bcast(first, 1) != 0;
    if (e.dag && !done1) sides |= ordb & 0xFu;
    // trace only: sweep history of the exact method, inflow sides and flags
    unsigned long long hist = e.trace ? ((unsigned long long)sides << 60 | (unsigned long long)fl << 56 |
                                         (unsigned long long)is_first << 55)
                                      : 0ull;
    order_acquire();
    if constexpr (HEAP) heap_fix(e, g >> 6, lane);  // g is running now
    tick(e, ph, kPhClaim, &t0);
    if (e.trace) tr[3] = wall_clock64();
    // a cell's interior is written only by its own processing
    tile_load(I, B, g, true, e.dag && is_first && !(ordb & kOrdSource));
    T pub[4];
    pub[0] = lane < B.hgt ? tu[(lane + 1) * P + 1] : inf_v<T>();
    pub[1] = lane < B.hgt ? tu[(lane + 1) * P + B.w] : inf_v<T>();
    pub[2] = lane < B.w ? tu[P + lane + 1] : inf_v<T>();
    pub[3] = lane < B.w ? tu[B.hgt * P + lane + 1] : inf_v<T>();
    tick(e, ph, kPhLoad, &t0);
    if (e.trace) tr[1] = wall_clock64();
    bool aborted = false;
    for (;;) {
      if constexpr (M == kFmsm) {
        if (ordb & kOrdConverge) {
          // cells holding exit nodes (or unreached by the coarse front): plain
          // FSM to convergence
          for (int k = 0;; ++k) {
            const bool ch = sweep_tile<T, P, false>(tu, td, B.w, B.hgt, k & 3, lane) & 1u;
            if (ch) nsweeps++; else nchecks++;
            if (!ch || k > 4096) break;
          }
        } else {
          // at most four sweeps in the coarse-upwind directions, with
          // sweep-directional updates
          const uint32_t dirs = fmsm_dirs(ordb & 0xFu);
#pragma nounroll
          for (int d = 0; d < 4; ++d)
            if (dirs & (1u << d)) {
              const bool ch = sweep_tile<T, P, true>(tu, td, B.w, B.hgt, d, lane) & 1u;
              if (ch) nsweeps++; else nchecks++;
            }
        }
        tick(e, ph, kPhSweep, &t0);
      } else if constexpr (M == kFhcm) {
        // one non-directional sweep per flagged direction, canonical order
#pragma nounroll
        for (int d = 0; d < 4; ++d)
          if (fl & (1u << d)) {
            const bool ch = sweep_tile<T, P, false>(tu, td, B.w, B.hgt, d, lane) & 1u;
            if (ch) nsweeps++; else nchecks++;
          }
        tick(e, ph, kPhSweep, &t0);
        publish<T, P, M, (NW == 1)>(e, I, B, g, tu, td, hacc, pub, is_first, lane);
        is_first = false;
        tick(e, ph, kPhPublish, &t0);
      } else {
        // exact: the first sweep starts in a corner between two sides with
        // inflow (one-axis inflow: a corner of such a side), else in a
        // flagged direction.  Each further sweep reverses the axis along
        // which the last sweep left a node below its upwind neighbour (both
        // axes: x and y in turn); after eight sweeps the canonical cycle.
        // Until converged.  The order changes the work, not the result.
        const uint32_t lead = fmsm_dirs(sides);
        const uint32_t pick = lead ? lead : fl;
        int dir = pick ? __builtin_ctz(pick) : 0;
        bool flip_x_next = true;
        for (int k = 0;; ++k) {
          const uint32_t res = sweep_tile<T, P, false, false, true>(tu, td, B.w, B.hgt, dir, lane);
          const bool ch = res & 1u;
          if (ch) nsweeps++; else nchecks++;
          tick(e, ph, kPhSweep, &t0);
          if (e.eager && (ch || is_first)) {
            publish<T, P, M, (NW == 1)>(e, I, B, g, tu, td, hacc, pub, is_first, lane);
            is_first = false;
            tick(e, ph, kPhPublish, &t0);
          }
          if (e.trace && k < 11) hist |= (unsigned long long)(dir | (res << 2)) << (5 * k);
          if (!(res & 6u)) break;  // no change, or no backflow: converged
          if (k > 4096) {  // a cell solve always terminates; guard anyway
            if (lane == 0) set_err(ctl, kErrGuard);
            aborted = true;
            break;
          }
          // direction bits: x reversed by dir ^ 3, y reversed by dir ^ 1
          if (k >= 7) {
            dir = (k + 1) & 3;
          } else if ((res & 6u) == 6u) {
            dir ^= flip_x_next ? 3 : 1;
            flip_x_next = !flip_x_next;
          } else if (res & 2u) {
            dir ^= 3;
            flip_x_next = false;
          } else {
            dir ^= 1;
            flip_x_next = true;
          }
        }
        if (!e.eager) {
          publish<T, P, M, (NW == 1)>(e, I, B, g, tu, td, hacc, pub, is_first, lane);
          is_first = false;
          tick(e, ph, kPhPublish, &t0);
        }
      }
      if (aborted) break;
      if (e.trace && !tr[2]) tr[2] = wall_clock64();
      if constexpr (M != kFmsm) {
        // publish has made the boundary visible: later neighbours start
        // while the interior is written back
        if (lane < 4 && e.dag && !__builtin_amdgcn_readfirstlane(done1))  // lane 0's flag
          release_later<(NW == 1)>(e, g, I, B, ordb, lane);
      }
      tile_store(I, B, g);
      order_release();
      int again = 0;
      if (lane == 0) {
        if (e.dag && !done1) {
          if (M == kFmsm)
            for (int sd = 0; sd < 4; ++sd) release_later<(NW == 1)>(e, g, I, B, ordb, sd);
          done1 = 1;
        }
        uint32_t exp = run_state;
        const bool idle =
            M == kFmsm ||
            __hip_atomic_compare_exchange_strong(&e.st[g], &exp, kDone1, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (idle) {
          if (M == kFmsm) st_coh(&e.st[g], kDone1);
          cell_idle(e, g);
          q_done(e, ring);
        } else {
          // re-requested while running: take it again at once
          const uint32_t old = claim(e, g);
          run_state = (old & kDone1) | kRunning;
          fl = (old >> kFlagShift) & 0xFu;
          sides = (old >> kSideShift) & 0xFu;
          const uint32_t v = ld_coh(&e.visits[g]);
          st_coh(&e.visits[g], v + 1u);
          count_visit(e, I, g);
          again = 1;
        }
      }
      again = bcast(again, 0);
      tick(e, ph, kPhFinish, &t0);
      if (!again) {
        if constexpr (HEAP) {  // g is idle, its neighbours may be pending with lower keys
          const int kx = __builtin_amdgcn_readfirstlane(I.kx);
#pragma nounroll
          for (int x = 0; x < 5; ++x)
            heap_fix(e, (g + (x == 1 ? -1 : x == 2 ? 1 : x == 3 ? -kx : x == 4 ? kx : 0)) >> 6, lane);
        }
        break;
      }
      if (get_err(ctl)) break;
      fl = (uint32_t)bcast((int)fl, 0);
      sides = (uint32_t)bcast((int)sides, 0);
      done1 = 1;
      order_acquire();
      load_tile_v<T, P, 1, 2>(tu, td, I, B, lane, false, false, 0);  // fresh halo only
      halo_to_masks<T, P>(td, B.w, B.hgt, lane, hacc);
    }
    if (lane == 0) {
      if (NW == 1 && e.ninst > 1) {  // per-instance statistics of a batch (visits: count_visit)
        unsigned long long* is = e.istat + 4 * (size_t)inst_index(e, g);
        atomic_add_relaxed(is + 1, nsweeps - sw0);
        atomic_add_relaxed(is + 2, nchecks - ch0);
      }
      if (e.trace) {
        const unsigned int slot = atomic_add_relaxed(e.trace_n, 1u);
        if (slot < e.trace_cap) {
          unsigned long long* t = e.trace + (size_t)slot * 8;
          t[0] = (unsigned long long)g | (((nsweeps - sw0) & 0xffffull) << 32) |
                 (((nchecks - ch0) & 0xffffull) << 48);
          t[1] = e.ready_at[g];
          t[2] = tr[0];
          t[3] = tr[1];
          t[4] = tr[2];
          t[5] = wall_clock64();
          t[6] = hist;  // exact method: 5 bits per sweep (direction, result bits)
          t[7] = tr[3];
        }
      }
    }
    if (get_err(ctl)) break;
  }
  if (lane == 0) {
    // leaving while cells are still waiting, queued or running, with no
    // error recorded, can only be the time limit: the result is incomplete
    if (!get_err(ctl) && ld64(&ctl->active) != 0ull) set_err(ctl, kErrDeadline);
    atomic_add_relaxed(&ctl->sweeps, nsweeps);
    atomic_add_relaxed(&ctl->checks, nchecks);
    if (kProfiling && e.profile) {
      unsigned long long* c = &ctl->t_idle;  // t_idle .. t_finish in phase order
      for (int k = 0; k < kPhases; ++k) atomic_add_relaxed(c + k, ph[k]);
    }
  }
  }  // !get_err at entry
  if constexpr (NW > 1) {  // release the helper waves
    if (lane == 0) job.op = 0;
    __syncthreads();  // A
  }
}

// ----------------------------------------------------------------------------
// preparation kernels
// ----------------------------------------------------------------------------

__device__ __forceinline__ const Inst& inst_at(const Engine& e, int k) {
  return e.args_inst ? e.one : e.inst[k];
}

// Cell states, queue rings and control block.
__global__ void k_prep_cells(Engine e) {
  const int ninst = e.ninst;
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t c = tid; c < (size_t)e.ncells; c += stride) {
    // dependency ordering: the state's kRunning bit of a cell whose first
    // processing has not finished stays clear; kDone1 set means "idle"
    e.st[c] = e.dag ? 0u : kDone1;
    e.visits[c] = 0u;
    e.key[c] = kKeyInf;
    if (e.dag) {
      e.deps[c] = 0;
      e.ord[c] = 0;
    }
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
  // sequence 0: on the first lap a consumer waits for its producer (ticket
  // h waits for sequence h + 1 >= 1) and a producer does not look
  for (size_t k = tid; k < (size_t)e.q.nslot; k += stride) e.q.slot[k] = 0ull;
  for (size_t k = tid; k < 4 * (size_t)ninst; k += stride) e.istat[k] = 0ull;
  if (ninst > 1)
    for (size_t k = tid; k < (size_t)ninst; k += stride) e.iact[k] = 0ull;
  const size_t nctr = (size_t)e.q.nb * e.q.ng > e.q.nring ? (size_t)e.q.nb * e.q.ng : e.q.nring;
  for (size_t k = tid; k < nctr; k += stride) {
    e.q.head[k * kCtrStride] = 0ull;
    e.q.tail[k * kCtrStride] = 0ull;
    e.q.inflight[k * kCtrStride] = 0ull;
  }
  for (size_t k = tid; k < (size_t)e.q.ng; k += stride) {
    e.q.cursor[k * kCtrStride] = 0ull;
    e.q.queued[k * kCtrStride] = 0ull;
  }
  if (tid == 0 && e.q.ng > 1) {
    // one group of bands per problem, in problem order
    unsigned long long off = 0ull;
    for (int k = 0; k < ninst; ++k) {
      const Inst& I = e.inst[k];
      uint32_t cap = 1u;
      while (cap < (uint32_t)(I.kx * I.ky) + 1u) cap <<= 1;
      const double w = e.q.width > 0.0 ? e.q.width : e.q.width_cells * I.s * I.h;
      e.q.grp[k] = QGroup{off, cap, 0u, 1.0 / w, 0.0};
      off += (unsigned long long)cap * e.q.nb;
    }
  }
  if (tid == 0) {
    Ctl* c = e.ctl;
    c->active = ninst > 1 ? (unsigned long long)ninst : 0ull;  // problems / cells active
    c->visits = 0ull;
    c->sweeps = 0ull;
    c->checks = 0ull;
    c->band_steps = 0ull;
    c->mon_checks = 0ull;
    c->mon_ok = 0ull;
    c->err = 0u;
    c->t_idle = c->t_claim = c->t_load = c->t_sweep = c->t_publish = c->t_finish = 0ull;
    c->guard = e.guard;
    c->deadline = wall_clock64() + e.timeout_ticks;
  }
}

// delta = h/F on accessible nodes (validating F), +inf on obstacles; the
// first block of every problem also validates its exit nodes (index range,
// accessibility, finite q).
template <typename T>
__global__ void k_prep_nodes(Engine e) {
  const Inst I = inst_at(e, blockIdx.y);
  if (blockIdx.x == 0) {
    const long long nn = (long long)I.nx * I.ny;
    for (int s = threadIdx.x; s < I.nsrc; s += blockDim.x) {
      const long long k = I.src[s];
      const double q = I.q ? I.q[s] : 0.0;
      if (k < 0 || k >= nn || (I.mask && !I.mask[k]) || !isfinite(q)) set_err(e.ctl, kErrSource);
    }
  }
  const size_t n = (size_t)I.nx * I.ny;
  const T* F = static_cast<const T*>(I.F);
  const double* Fd = static_cast<const double*>(I.F);
  T* dl = static_cast<T*>(I.delta);
  const bool f64_input = I.qdense != nullptr;  // coarse problems carry double speeds
  bool bad = false;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x) {
    const bool acc = I.mask ? I.mask[k] != 0 : true;
    T d = inf_v<T>();
    if (acc) {
      const double f = f64_input ? Fd[k] : (double)F[k];
      if (!(f > 0.0) || !isfinite(f)) bad = true;
      d = (T)(I.h / f);
    }
    dl[k] = d;
  }
  if (bad) set_err(e.ctl, kErrSpeed);
}

__device__ __forceinline__ int cell_of_node(const Inst& I, int i, int j) {
  int cx = I.balanced ? (int)(((long long)i * I.kx) / I.nx) : i / I.s;
  int cy = I.balanced ? (int)(((long long)j * I.ky) / I.ny) : j / I.s;
  if (cx >= I.kx) cx = I.kx - 1;
  if (cy >= I.ky) cy = I.ky - 1;
  while (cx > 0 && cell_lo(cx, I.nx, I.kx, I.s, I.balanced) > i) cx--;
  while (cx + 1 < I.kx && cell_lo(cx + 1, I.nx, I.kx, I.s, I.balanced) <= i) cx++;
  while (cy > 0 && cell_lo(cy, I.ny, I.ky, I.s, I.balanced) > j) cy--;
  while (cy + 1 < I.ky && cell_lo(cy + 1, I.ny, I.ky, I.s, I.balanced) <= j) cy++;
  return I.cell0 + cy * I.kx + cx;
}

// u = +inf, or the dense exit costs (coarse problems: those nodes are frozen
// and, without dependency ordering, their cells queued).  A pass of its own
// after k_prep_nodes: u is often the caller's output, which a problem that
// fails validation leaves untouched.
template <typename T>
__global__ void k_init_u(Engine e) {
  if (get_err(e.ctl)) return;
  const Inst I = inst_at(e, blockIdx.y);
  const size_t n = (size_t)I.nx * I.ny;
  T* u = static_cast<T*>(I.u);
  T* dl = static_cast<T*>(I.delta);
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x) {
    T v = inf_v<T>();
    if (I.qdense && I.qdense[k] < __builtin_huge_val() && (!I.mask || I.mask[k])) {
      v = (T)I.qdense[k];
      dl[k] = inf_v<T>();
      if (!e.dag) {
        const int g = cell_of_node(I, (int)(k % I.nx), (int)(k / I.nx));
        __hip_atomic_fetch_min(&e.key[g], key_bits((double)v), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        requeue(e, g, e.method == kFhcm ? 0xFu : 0u, 0u, (double)v);
      }
    }
    u[k] = v;
  }
}

__device__ __forceinline__ void atomic_min_val(double* p, double v) {
  unsigned long long* a = reinterpret_cast<unsigned long long*>(p);
  unsigned long long old = ld_coh(a);
  while (__builtin_bit_cast(double, old) > v) {
    if (__hip_atomic_compare_exchange_strong(a, &old, __builtin_bit_cast(unsigned long long, v),
                                             __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      break;
  }
}
__device__ __forceinline__ void atomic_min_val(float* p, float v) {
  unsigned int* a = reinterpret_cast<unsigned int*>(p);
  unsigned int old = ld_coh(a);
  while (__builtin_bit_cast(float, old) > v) {
    if (__hip_atomic_compare_exchange_strong(a, &old, __builtin_bit_cast(unsigned int, v),
                                             __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      break;
  }
}

// u = min q at sources, sources frozen (delta = +inf), and -- unless cells
// are ordered by dependency counts -- their cells queued (Algorithm
// generic_LC_cells, cell and fine-grid initialisation; Algorithm FHCM for the
// key 0 and four raised directions).
template <typename T>
__global__ void k_apply_sources(Engine e) {
  if (get_err(e.ctl)) return;
  const Inst I = inst_at(e, blockIdx.y);
  if (I.qdense) return;
  T* u = static_cast<T*>(I.u);
  T* dl = static_cast<T*>(I.delta);
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < I.nsrc; s += gridDim.x * blockDim.x) {
    const long long k = I.src[s];
    const double q = I.q ? I.q[s] : 0.0;
    atomic_min_val(u + k, (T)q);
    dl[k] = inf_v<T>();
    if (e.dag) continue;
    const int g = cell_of_node(I, (int)(k % I.nx), (int)(k / I.nx));
    const double key = e.method == kFhcm ? 0.0 : q;
    __hip_atomic_fetch_min(&e.key[g], key_bits(key), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    requeue(e, g, e.method == kFhcm ? 0xFu : 0u, 0u, key);
  }
}

// Coarse grid inputs (FMSM Part I, Section 3.1: a coarse gridpoint is the
// centre of its cell): per cell the speed at the centre -- the centre node,
// or the mean of the accessible nodes around it -- falling back to the mean
// speed over the cell's accessible nodes; whether it has an accessible node;
// and (initially +inf) the smallest exit cost of its exit nodes.  One wave
// per cell: lane l sums column l bottom to top (loads of a row are
// contiguous), then lane 0 adds the column sums left to right -- a fixed
// order the CPU oracle uses as well.
template <typename T>
__global__ __launch_bounds__(64) void k_coarse_cells(Engine e, const CoarseOut* co) {
  __shared__ double csum[64];
  __shared__ int ccnt[64];
  const int lane = threadIdx.x;
  for (int g = blockIdx.x; g < e.ncells; g += gridDim.x) {
    const int k = inst_index(e, g);
    const Inst I = inst_at(e, k);
    const CellBox B = cell_box(I, g - I.cell0);
    const T* F = static_cast<const T*>(I.F);
    // the speed at the cell centre: the centre node, or the mean of the
    // accessible nodes around it (x ascending, then y); an accessible one
    // also makes the cell accessible, so the cell mean is needed only when
    // none of them is
    double sc = 0.0;
    int nc = 0;
    if (lane == 0) {
      const int ia = (B.x0 + B.x1 - 1) / 2, ib = (B.x0 + B.x1) / 2;
      const int ja = (B.y0 + B.y1 - 1) / 2, jb = (B.y0 + B.y1) / 2;
      for (int a = 0; a < (ia == ib ? 1 : 2); ++a)
        for (int b = 0; b < (ja == jb ? 1 : 2); ++b) {
          const size_t n = (size_t)(b ? jb : ja) * I.nx + (a ? ib : ia);
          if (I.mask && !I.mask[n]) continue;
          sc += (double)F[n];
          nc++;
        }
    }
    nc = __builtin_amdgcn_readfirstlane(nc);
    const int cl = g - I.cell0;
    if (nc > 0) {
      if (lane == 0) {
        co[k].F[cl] = sc / nc;
        co[k].mask[cl] = 1;
        co[k].q[cl] = __builtin_huge_val();
      }
      continue;
    }
    // no accessible centre node: the mean of F over the cell, summed column
    // by column (each column bottom to top, then the columns left to right)
    double col = 0.0;
    int cnt = 0;
    if (lane < B.w) {
#pragma unroll 16
      for (int j = B.y0; j < B.y1; ++j) {
        const size_t n = (size_t)j * I.nx + B.x0 + lane;
        const bool acc = !I.mask || I.mask[n];
        const double f = (double)F[n];
        if (acc) {
          col += f;
          cnt++;
        }
      }
    }
    csum[lane] = col;
    ccnt[lane] = cnt;
    __syncthreads();
    if (lane == 0) {
      double sum = 0.0;
      int c = 0;
      for (int l = 0; l < B.w; ++l) {
        sum += csum[l];
        c += ccnt[l];
      }
      co[k].F[cl] = c ? sum / c : 1.0;
      co[k].mask[cl] = c > 0;
      co[k].q[cl] = __builtin_huge_val();
    }
    __syncthreads();
  }
}

__global__ void k_coarse_sources(Engine e, const CoarseOut* co) {
  if (get_err(e.ctl)) return;  // an invalid exit node has no cell
  const int k = blockIdx.y;
  const Inst I = inst_at(e, k);
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < I.nsrc; s += gridDim.x * blockDim.x) {
    const long long n = I.src[s];
    if (n < 0 || n >= (long long)I.nx * I.ny) continue;  // reported by k_prep_nodes
    const double q = I.q ? I.q[s] : 0.0;
    const int g = cell_of_node(I, (int)(n % I.nx), (int)(n / I.nx));
    atomic_min_val(co[k].q + (g - I.cell0), q);
  }
}

// Fast Marching on the grid of cell centres (FMSM Part I, Section 3.1; the
// method of Section 2): one wave per problem.  Every exit cell is accepted
// first; their neighbours are then relaxed exit cell by exit cell in
// (q, index) order, and after that the smallest (value, index) entry of the
// front is accepted, one at a time, and its neighbours relaxed.  The four
// neighbours of a cell are pairwise non-adjacent, so four lanes relax them at
// once with the same result as one after the other.  The front is an
// unordered array of cells; each acceptance takes a wave-wide argmin over it.
// Values, step sizes, cell states and the front live in LDS when the coarse
// grid fits (lds_cells: 16-bit states and front entries, front values read
// through the front's cell index), else in the spill workspace (32-bit, with
// a copy of the front values next to the front).
constexpr int kFmmFar = -1, kFmmObst = -2, kFmmAcc = -3;

// FV: the spill layout (global memory, front values kept beside the front).
// In the LDS layout every access inside the acceptance loop is an LDS access
// of this one wave, which the LDS performs in order, so lanes see each
// other's writes without waiting (the acceptance ranks go to global memory
// and are never read back); the spill layout waits for its global accesses.
template <typename IdxT, bool FV>
__device__ void coarse_fmm(const CoarseOut& C, int kx, int ky, double hc, int lane, double* V,
                           double* dl, double* fv, IdxT* st, IdxT* fi) {
  const int J = kx * ky;
  const double INF = __builtin_huge_val();
  auto step_sync = [] {
    if constexpr (FV) {
      __syncthreads();
    } else {
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
  };
  for (int c = lane; c < J; c += 64) {
    const bool acc = C.mask[c] != 0;
    const double q = C.q[c];
    const bool exit = acc && q < INF;
    V[c] = exit ? q : INF;
    dl[c] = acc ? hc / C.F[c] : INF;
    st[c] = (IdxT)(!acc ? kFmmObst : exit ? kFmmAcc : kFmmFar);
    C.rank[c] = J + c;  // cells the front never reaches: after all others, by index
  }
  __syncthreads();
  // exit cells into the top of the front arrays, [J - ns, J)
  int ns = 0;
  for (int base = 0; base < J; base += 64) {
    const int c = base + lane;
    const bool is = c < J && st[c] == kFmmAcc;
    const unsigned long long m = ballot(is);
    if (is) {
      const int slot = J - 1 - ns - (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                                  __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
      if constexpr (FV) fv[slot] = V[c];
      fi[slot] = (IdxT)c;
    }
    ns += __builtin_popcountll(m);
  }
  __syncthreads();
  int nf = 0, na = 0, rs = ns;
  for (;;) {
    const bool exits = rs > 0;
    const int lo = exits ? J - rs : 0, hi = exits ? J : nf;
    if (lo == hi) break;
    // accept the (value, index) minimum of [lo, hi); each lane takes four of
    // its slots per round so that their loads are in flight together
    double bv = INF;
    int bc = 0x7fffffff, bs = -1;
    for (int t0 = lo + lane; t0 < hi; t0 += 256) {
      int cq[4];
      double vq[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) cq[u] = t0 + 64 * u < hi ? (int)fi[t0 + 64 * u] : 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) vq[u] = t0 + 64 * u < hi ? (FV ? fv[t0 + 64 * u] : V[cq[u]]) : INF;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool take = t0 + 64 * u < hi && (vq[u] < bv || (vq[u] == bv && cq[u] < bc));
        bv = take ? vq[u] : bv;
        bc = take ? cq[u] : bc;
        bs = take ? t0 + 64 * u : bs;
      }
    }
    wave::argmin(bv, bc, bs, lane);
    if (lane == 0) {
      if (exits) {  // the exit list shrinks from below
        if constexpr (FV) fv[bs] = fv[lo];
        fi[bs] = fi[lo];
      } else {
        const int last = nf - 1;
        if (bs != last) {
          const int mv = fi[last];
          if constexpr (FV) fv[bs] = fv[last];
          fi[bs] = (IdxT)mv;
          st[mv] = (IdxT)bs;
        }
        st[bc] = (IdxT)kFmmAcc;
      }
      to_global(C.rank)[bc] = na;  // a global store: LDS waits do not wait for it
    }
    if (exits) rs--;
    else nf--;
    na++;
    step_sync();
    // relax the four neighbours W, E, S, N of the accepted cell
    const int cx = bc % kx, cy = bc / kx;
    const int nx = cx + (lane == 0 ? -1 : lane == 1 ? 1 : 0);
    const int ny = cy + (lane == 2 ? -1 : lane == 3 ? 1 : 0);
    const bool inb = lane < 4 && nx >= 0 && nx < kx && ny >= 0 && ny < ky;
    // every load of the relaxation at once (indices outside the grid are
    // replaced by the accepted cell's and their values by +inf)
    const int nb = inb ? ny * kx + nx : bc;
    const int sn = inb ? (int)st[nb] : kFmmObst;
    const double vW = V[inb && nx > 0 ? nb - 1 : bc], vE = V[inb && nx + 1 < kx ? nb + 1 : bc];
    const double vS = V[inb && ny > 0 ? nb - kx : bc], vN = V[inb && ny + 1 < ky ? nb + kx : bc];
    const double dn = dl[nb], v0 = V[nb];
    const bool live = inb && sn != kFmmObst && sn != kFmmAcc;
    double vn = INF;
    if (live) {
      const double uW = nx > 0 ? vW : INF, uE = nx + 1 < kx ? vE : INF;
      const double uS = ny > 0 ? vS : INF, uN = ny + 1 < ky ? vN : INF;
      const double a = uW < uE ? uW : uE, b = uS < uN ? uS : uN;
      const double t = (a < b ? a : b) == INF ? INF : local_update(a, b, dn);
      vn = v0;
      if (t < vn) {
        vn = t;
        V[nb] = t;
      }
      if constexpr (FV)
        if (sn >= 0) fv[sn] = vn;
    }
    const bool push = live && sn == kFmmFar;
    const unsigned long long m = ballot(push);
    if (push) {
      const int slot = nf + (int)__builtin_amdgcn_mbcnt_lo((unsigned)m, 0u);
      if constexpr (FV) fv[slot] = vn;
      fi[slot] = (IdxT)nb;
      st[nb] = (IdxT)slot;
    }
    nf += __builtin_popcountll(m);
    step_sync();
  }
}

// Exact solve of a coarse grid of at most kCoarseJacobiMax cells by Jacobi
// iteration, one workgroup per problem, NPT cells per thread (1 up to 1024
// cells, else kCoarseJacobiPer with 1024 threads): every iteration applies
// the local update of Section 2 to all cells at once from the previous
// iterate (two LDS buffers, one barrier per iteration) until no value
// decreases.  The update is causal (a new value exceeds the values it is
// computed from), so a value is final once the chain of cells it depends on
// is, and at most J + 1 iterations are needed.  The exact, HCM and FHCM
// methods use these values only to order the fine cells.
template <int NPT>
__global__ __launch_bounds__(1024) void k_coarse_jacobi(Engine e, const CoarseOut* co) {
  __shared__ double ub[2][1024 * NPT];
  __shared__ int dec_any[3];  // iteration it reports decreases in dec_any[it % 3]
  const int k = blockIdx.x;
  const Inst I = inst_at(e, k);
  const CoarseOut C = co[k];
  const int kx = I.kx, ky = I.ky, J = kx * ky;
  const double hc = (double)I.s * I.h;
  const double inf = __builtin_huge_val();
  // dl = h^c / F^c on coarse cells that are updated: accessible and not exit cells
  double dl[NPT], u[NPT];
  int cx[NPT], cy[NPT];
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int c = threadIdx.x + m * (int)blockDim.x;
    dl[m] = inf;
    u[m] = inf;
    cx[m] = cy[m] = 0;
    if (c < J) {
      cx[m] = c % kx;
      cy[m] = c / kx;
      if (C.mask[c]) {
        u[m] = C.q[c];
        if (!(u[m] < inf)) dl[m] = hc / C.F[c];
      }
      ub[0][c] = u[m];
    }
  }
  if (threadIdx.x < 3) dec_any[threadIdx.x] = 0;
  __syncthreads();
  for (int it = 0; it <= J; ++it) {
    const double* cur = ub[it & 1];
    double* nxt = ub[(it + 1) & 1];
    bool dec = false;
#pragma unroll
    for (int m = 0; m < NPT; ++m) {
      const int c = threadIdx.x + m * (int)blockDim.x;
      if (c < J && dl[m] < inf) {
        const double l = cx[m] > 0 ? cur[c - 1] : inf, r = cx[m] + 1 < kx ? cur[c + 1] : inf;
        const double d = cy[m] > 0 ? cur[c - kx] : inf, t = cy[m] + 1 < ky ? cur[c + kx] : inf;
        const double a = l < r ? l : r, b = d < t ? d : t;
        const double v = local_update(a, b, dl[m]);
        if (v < u[m]) {
          u[m] = v;
          dec = true;
        }
      }
      if (c < J) nxt[c] = u[m];
    }
    // the flag of iteration it + 1 was last read after the barrier of
    // iteration it - 2, which every thread has passed
    const int f = it % 3;
    if (threadIdx.x == 0) dec_any[f == 2 ? 0 : f + 1] = 0;
    if (dec) dec_any[f] = 1;
    __syncthreads();
    if (!dec_any[f]) break;
  }
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int c = threadIdx.x + m * (int)blockDim.x;
    if (c < J) C.u[c] = u[m];
  }
}

__global__ __launch_bounds__(64) void k_coarse_fmm(Engine e, const CoarseOut* co, int lds_cells,
                                                   FmmSpill spill) {
  extern __shared__ __align__(16) unsigned char fmm_lds[];
  const int k = blockIdx.x;
  const Inst I = inst_at(e, k);
  const CoarseOut C = co[k];
  const int lane = threadIdx.x, J = I.kx * I.ky;
  const double hc = (double)I.s * I.h;
  if (J <= lds_cells) {  // lds_cells < 2^15: states and front entries fit 16 bits
    double* V = reinterpret_cast<double*>(fmm_lds);
    double* dl = V + J;
    int16_t* st = reinterpret_cast<int16_t*>(dl + J);
    int16_t* fi = st + J;
    coarse_fmm<int16_t, false>(C, I.kx, I.ky, hc, lane, V, dl, nullptr, st, fi);
    for (int c = lane; c < J; c += 64) C.u[c] = V[c];
  } else {
    coarse_fmm<int32_t, true>(C, I.kx, I.ky, hc, lane, C.u, spill.delta + I.cell0,
                              spill.fval + I.cell0, spill.st + I.cell0, spill.fidx + I.cell0);
  }
}

// Order of the cells: exit cells first by (q, index), then by (coarse value,
// index) -- the acceptance order of Fast Marching on the coarse grid -- and
// cells the coarse front does not reach last, by index.  Each cell counts
// the accessible neighbours that precede it; a cell with none is queued.
__global__ void k_dag(Engine e, const CoarseOut* co) {
  const int lane = threadIdx.x & 63;
  // uniform trip count: every lane of a wave takes part in the aggregation
  for (int g0 = blockIdx.x * blockDim.x; g0 < e.ncells; g0 += gridDim.x * blockDim.x) {
    const int g = g0 + (int)threadIdx.x;
    int k = -1, n = 0;
    if (g < e.ncells) {
      k = inst_index(e, g);
      const Inst I = inst_at(e, k);
      const CoarseOut C = co[k];
      const int c = g - I.cell0;
      if (!C.mask[c]) {
        e.ord[g] = kOrdEmpty;
        e.st[g] = kDone1;
        k = -1;
      } else {
        auto cls = [&](int x) { return C.q[x] < __builtin_huge_val() ? 0 : 1; };
        auto val = [&](int x) { return C.q[x] < __builtin_huge_val() ? C.q[x] : C.u[x]; };
        auto before = [&](int x, int y) {  // does cell x precede cell y?
          if (C.rank) return C.rank[x] < C.rank[y];
          const int cxx = cls(x), cyy = cls(y);
          if (cxx != cyy) return cxx < cyy;
          const double vx = val(x), vy = val(y);
          if (vx != vy) return vx < vy;
          return x < y;
        };
        const int cx = c % I.kx, cy = c / I.kx;
        uint8_t o = (cls(c) == 0 || !(val(c) < __builtin_huge_val())) ? kOrdConverge : 0;
        if (cls(c) == 0) o |= kOrdSource;
        for (int side = 0; side < 4; ++side) {
          int nb = -1;
          if (side == 0 && cx > 0) nb = c - 1;
          if (side == 1 && cx + 1 < I.kx) nb = c + 1;
          if (side == 2 && cy > 0) nb = c - I.kx;
          if (side == 3 && cy + 1 < I.ky) nb = c + I.kx;
          if (nb < 0 || !C.mask[nb]) continue;
          if (before(nb, c)) {
            o |= (uint8_t)(1u << side);
            n++;
          }
        }
        e.ord[g] = o;
        e.deps[g] = n;
      }
    }
    // the active counts (cell_active) of the wave's accessible cells: one
    // atomic per problem among them instead of one per cell, all before any
    // of them is queued (the solver starts after this kernel)
    unsigned long long todo = ballot(k >= 0);
    while (todo) {
      const int leader = __builtin_ctzll(todo);
      const int kl = __shfl(k, leader, 64);
      const unsigned long long same = ballot(k == kl);
      if (lane == leader) {
        const unsigned long long cnt = (unsigned long long)__builtin_popcountll(same);
        if (e.ninst > 1) atomic_add_relaxed(&e.iact[kl], cnt);
        else atomic_add_relaxed(&e.ctl->active, cnt);
      }
      todo &= ~same;
    }
    if (k >= 0 && n == 0 && !get_err(e.ctl)) release_first(e, g);
  }
}

// Whole-grid sweeping (Algorithm FSM; Locking Sweeping with tile locks):
// the tiles of one anti-diagonal of sweep ordering `dir`, one wave each.
// Tiles on one anti-diagonal share no side, and every tile upwind of a tile
// lies on an earlier anti-diagonal (an earlier launch), so the launches of
// one sweep reproduce the serial lexicographic sweep bit for bit.
template <typename T, int S>
__global__ __launch_bounds__(64) void k_sweep_diag(Engine e, SweepArgs a) {
  constexpr int P = S + 2;
  __shared__ T tu_mem[TileLds<P>::kSize];
  T* const tu = tu_mem + TileLds<P>::kBefore;
  __shared__ T td[P * P];
  const int lane = threadIdx.x;
  if (get_err(e.ctl)) return;
  const Inst I = inst_at(e, 0);
  const int sx = (a.dir == 0 || a.dir == 1) ? 1 : -1;
  const int sy = (a.dir == 0 || a.dir == 3) ? 1 : -1;
  const int ta = (a.diag - (I.ky - 1) > 0 ? a.diag - (I.ky - 1) : 0) + (int)blockIdx.x;
  const int tb = a.diag - ta;
  if (ta >= I.kx || tb < 0 || tb >= I.ky) return;
  const int cx = sx > 0 ? ta : I.kx - 1 - ta;
  const int cy = sy > 0 ? tb : I.ky - 1 - tb;
  const int g = cy * I.kx + cx;
  if (a.locking && !a.dirty[g]) {
    if (lane == 0) atomic_add_relaxed(&a.stat[3], 1ull);
    return;
  }
  const CellBox B = cell_box(I, g);
  load_tile<T, P>(tu, td, I, B, lane, true);
  halo_to_masks<T, P>(td, B.w, B.hgt, lane, nullptr);
  double mx = 0.0;
  int cnt = 0;
  sweep_tile<T, P, false, true>(tu, td, B.w, B.hgt, a.dir, lane, &mx, &cnt);
  for (int off = 32; off > 0; off >>= 1) {
    const double om = __shfl_xor(mx, off, 64);
    mx = om > mx ? om : mx;
    cnt += __shfl_xor(cnt, off, 64);
  }
  if (cnt) store_tile<T, P>(tu, I, B, lane);
  if (lane == 0) {
    // a non-negative double orders like its bit pattern
    __hip_atomic_fetch_max(&a.stat[0], __builtin_bit_cast(unsigned long long, mx), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    atomic_add_relaxed(&a.stat[1], (unsigned long long)cnt);
    atomic_add_relaxed(&a.stat[2], 1ull);
    if (a.locking) {
      a.dirty[g] = cnt ? 1 : 0;
      if (cnt) {
        if (cx > 0) a.dirty[g - 1] = 1;
        if (cx + 1 < I.kx) a.dirty[g + 1] = 1;
        if (cy > 0) a.dirty[g - I.kx] = 1;
        if (cy + 1 < I.ky) a.dirty[g + I.kx] = 1;
      }
    }
  }
}

// Locking start: the tiles holding exit nodes and their neighbours may
// change (every other tile is +inf with a +inf halo).
__global__ void k_sweep_seed(Engine e, uint8_t* dirty) {
  const Inst I = inst_at(e, 0);
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < I.nsrc; s += gridDim.x * blockDim.x) {
    const long long k = I.src[s];
    if (k < 0 || k >= (long long)I.nx * I.ny) continue;  // reported by k_prep_nodes
    const int g = cell_of_node(I, (int)(k % I.nx), (int)(k / I.nx));
    const int cx = g % I.kx, cy = g / I.kx;
    dirty[g] = 1;
    if (cx > 0) dirty[g - 1] = 1;
    if (cx + 1 < I.kx) dirty[g + 1] = 1;
    if (cy > 0) dirty[g - I.kx] = 1;
    if (cy + 1 < I.ky) dirty[g + I.kx] = 1;
  }
}

// Fixed-point residual max |T(u)_k - u_k| / u_k in FP64 over accessible,
// non-exit nodes with finite u (inf where u is inf but T(u) is finite).
template <typename T>
__global__ void k_residual(Engine e, int inst0) {
  const int ki = inst0 + (int)blockIdx.y;
  const Inst I = inst_at(e, ki);
  const T* u = static_cast<const T*>(I.u);
  const T* F = static_cast<const T*>(I.F);
  const T* dl = static_cast<const T*>(I.delta);
  const size_t n = (size_t)I.nx * I.ny;
  double mx = 0.0;
  for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (size_t)gridDim.x * blockDim.x) {
    if (dl[k] == inf_v<T>()) continue;  // obstacle or exit node
    const int i = (int)(k % I.nx), j = (int)(k / I.nx);
    const double INF = __builtin_huge_val();
    const double uW = i > 0 ? (double)u[k - 1] : INF;
    const double uE = i + 1 < I.nx ? (double)u[k + 1] : INF;
    const double uS = j > 0 ? (double)u[k - I.nx] : INF;
    const double uN = j + 1 < I.ny ? (double)u[k + I.nx] : INF;
    const double a = uW < uE ? uW : uE, b = uS < uN ? uS : uN;
    double t = local_update(a, b, I.h / (double)F[k]);
    if (t != t) t = INF;
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
    __hip_atomic_fetch_max(&e.istat[4 * (size_t)ki + 3],
                           __builtin_bit_cast(unsigned long long, mx), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

template <typename S, typename D>
__global__ void k_convert(const S* src, D* dst, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    dst[k] = (D)src[k];
}

// Latency of the sweep's dependent chain: one wave alone sweeps one S x S
// tile in LDS `sweeps` times (direction SW; exit node at the south-west
// corner, +inf elsewhere, so every sweep runs the same branch-free steps as
// in the exact method's solver) and reports the wall-clock ticks of the loop.
// One sweep is 2S - 1 anti-diagonal steps, each one dependent local update
// per lane.
template <typename T, int S>
__global__ __launch_bounds__(64) void k_probe_sweep(int sweeps, unsigned long long* ticks) {
  constexpr int P = S + 2;
  __shared__ T tu_mem[TileLds<P>::kSize];
  T* const tu = tu_mem + TileLds<P>::kBefore;
  __shared__ T td[P * P];
  const int lane = threadIdx.x;
  for (int k = lane; k < P * P; k += 64) {
    tu[k] = inf_v<T>();
    td[k] = (T)(1.0 / S);
  }
  __syncthreads();
  halo_to_masks<T, P>(td, S, S, lane, nullptr);
  __syncthreads();
  if (lane == 0) tu[P + 1] = (T)0;  // the exit node
  __syncthreads();
  const unsigned long long t0 = wall_clock64();
  uint32_t acc = 0;
  for (int r = 0; r < sweeps; ++r) acc += sweep_tile<T, P, false, false, true>(tu, td, S, S, 0, lane);
  const unsigned long long t1 = wall_clock64();
  if (lane == 0) ticks[0] = (t1 - t0) | ((unsigned long long)(acc & 1u) << 63);
}

}  // namespace

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------

hipError_t launch_probe_sweep(int dtype, int side, int sweeps, unsigned long long* ticks,
                              hipStream_t stream) {
  if (dtype == 0 && side == 64)
    hipLaunchKernelGGL((k_probe_sweep<double, 64>), dim3(1), dim3(64), 0, stream, sweeps, ticks);
  else if (dtype == 0 && side == 32)
    hipLaunchKernelGGL((k_probe_sweep<double, 32>), dim3(1), dim3(64), 0, stream, sweeps, ticks);
  else if (dtype == 1 && side == 64)
    hipLaunchKernelGGL((k_probe_sweep<float, 64>), dim3(1), dim3(64), 0, stream, sweeps, ticks);
  else if (dtype == 1 && side == 32)
    hipLaunchKernelGGL((k_probe_sweep<float, 32>), dim3(1), dim3(64), 0, stream, sweeps, ticks);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

static int grid_for(int64_t n, int block, int cap) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

hipError_t launch_prepare(const Engine& e, int64_t max_nodes, hipStream_t stream) {
  const int gy = e.ninst;
  const int64_t cwork = (int64_t)e.ncells > (int64_t)e.q.nslot ? (int64_t)e.ncells : (int64_t)e.q.nslot;
  hipLaunchKernelGGL(k_prep_cells, dim3(grid_for(cwork, 256, 4096)), dim3(256), 0, stream, e);
  // per problem of a batch at most 128 blocks (grid-stride): with 512 most
  // blocks of the small problems found no node (256-instance batch:
  // 3.65 -> 3.57 ms per batch)
  const dim3 gn(grid_for(max_nodes, 256, gy > 1 ? 128 : 8192), gy);
  if (e.dtype == 0) hipLaunchKernelGGL(k_prep_nodes<double>, gn, dim3(256), 0, stream, e);
  else hipLaunchKernelGGL(k_prep_nodes<float>, gn, dim3(256), 0, stream, e);
  if (e.dtype == 0) hipLaunchKernelGGL(k_init_u<double>, gn, dim3(256), 0, stream, e);
  else hipLaunchKernelGGL(k_init_u<float>, gn, dim3(256), 0, stream, e);
  if (e.dtype == 0) hipLaunchKernelGGL(k_apply_sources<double>, dim3(1, gy), dim3(64), 0, stream, e);
  else hipLaunchKernelGGL(k_apply_sources<float>, dim3(1, gy), dim3(64), 0, stream, e);
  return hipGetLastError();
}

template <typename T, int M, int NW, bool HEAP = false>
static void launch_solve_w(const Engine& e, dim3 g, int tile, hipStream_t stream) {
  if (tile <= 16) hipLaunchKernelGGL((k_solve<T, 16, M, NW, HEAP>), g, dim3(64 * NW), 0, stream, e);
  else if (tile <= 32) hipLaunchKernelGGL((k_solve<T, 32, M, NW, HEAP>), g, dim3(64 * NW), 0, stream, e);
  else hipLaunchKernelGGL((k_solve<T, 64, M, NW, HEAP>), g, dim3(64 * NW), 0, stream, e);
}
// single problems: four waves per worker share the tile transfers; the heap
// schedule: one single-wave worker
template <typename T, int M>
static void launch_solve_t(const Engine& e, dim3 g, int tile, hipStream_t stream) {
  if constexpr (M != kFmsm)
    if (e.heap) return launch_solve_w<T, M, 1, true>(e, g, tile, stream);
  if (e.ninst == 1) launch_solve_w<T, M, kSolveWaves1>(e, g, tile, stream);
  else launch_solve_w<T, M, 1>(e, g, tile, stream);
}

template <typename T>
static void launch_solve_m(const Engine& e, dim3 g, int tile, hipStream_t stream) {
  if (e.method == kFmsm) launch_solve_t<T, kFmsm>(e, g, tile, stream);
  else if (e.method == kFhcm) launch_solve_t<T, kFhcm>(e, g, tile, stream);
  else launch_solve_t<T, kExact>(e, g, tile, stream);
}

template <typename T, int M>
static int occupancy_t(int tile) {
  int n = 0;
  hipError_t err;
  if (tile <= 16)
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_solve<T, 16, M, 1>, 64, 0);
  else if (tile <= 32)
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_solve<T, 32, M, 1>, 64, 0);
  else
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_solve<T, 64, M, 1>, 64, 0);
  return err == hipSuccess && n > 0 ? n : 1;
}

int solve_waves_per_cu(int dtype, int method, int tile) {
  if (dtype == 0) {
    if (method == kFmsm) return occupancy_t<double, kFmsm>(tile);
    if (method == kFhcm) return occupancy_t<double, kFhcm>(tile);
    return occupancy_t<double, kExact>(tile);
  }
  if (method == kFmsm) return occupancy_t<float, kFmsm>(tile);
  if (method == kFhcm) return occupancy_t<float, kFhcm>(tile);
  return occupancy_t<float, kExact>(tile);
}

hipError_t launch_solve(const Engine& e, int workers, int tile, hipStream_t stream) {
  const dim3 g(workers);
  if (e.dtype == 0) launch_solve_m<double>(e, g, tile, stream);
  else launch_solve_m<float>(e, g, tile, stream);
  return hipGetLastError();
}

hipError_t launch_residual(const Engine& e, int64_t max_nodes, hipStream_t stream, int inst0,
                           int count) {
  const int n = count > 0 ? count : e.ninst;
  const dim3 gn(grid_for(max_nodes, 256, n > 1 ? 256 : 4096), n);
  if (e.dtype == 0) hipLaunchKernelGGL(k_residual<double>, gn, dim3(256), 0, stream, e, inst0);
  else hipLaunchKernelGGL(k_residual<float>, gn, dim3(256), 0, stream, e, inst0);
  return hipGetLastError();
}

hipError_t launch_coarse_inputs(const Engine& fine, const CoarseOut* co_dev, int max_src,
                                hipStream_t stream) {
  const dim3 gc(fine.ncells < 65535 ? fine.ncells : 65535);
  if (fine.dtype == 0) hipLaunchKernelGGL(k_coarse_cells<double>, gc, dim3(64), 0, stream, fine, co_dev);
  else hipLaunchKernelGGL(k_coarse_cells<float>, gc, dim3(64), 0, stream, fine, co_dev);
  hipLaunchKernelGGL(k_coarse_sources, dim3(grid_for(max_src, 64, 1024), fine.ninst), dim3(64), 0,
                     stream, fine, co_dev);
  return hipGetLastError();
}

int coarse_fmm_lds_cells() {
  static const int cells = [] {
    int dev = 0, lim = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      lim = 65536;
    if (lim > 65536 &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_coarse_fmm),
                            hipFuncAttributeMaxDynamicSharedMemorySize, lim) != hipSuccess)
      lim = 65536;
    const int c = lim / kFmmLdsBytesPerCell;
    return c < 32767 ? c : 32767;
  }();
  return cells;
}

hipError_t launch_sweep_diag(const Engine& e, const SweepArgs& a, int tiles, hipStream_t stream) {
  if (e.dtype == 0) hipLaunchKernelGGL((k_sweep_diag<double, kSweepTile>), dim3(tiles), dim3(64), 0, stream, e, a);
  else hipLaunchKernelGGL((k_sweep_diag<float, kSweepTile>), dim3(tiles), dim3(64), 0, stream, e, a);
  return hipGetLastError();
}

hipError_t launch_sweep_seed(const Engine& e, int nsrc, uint8_t* dirty, hipStream_t stream) {
  hipLaunchKernelGGL(k_sweep_seed, dim3(grid_for(nsrc, 256, 1024)), dim3(256), 0, stream, e, dirty);
  return hipGetLastError();
}

hipError_t launch_coarse_jacobi(const Engine& fine, const CoarseOut* co_dev, int max_cells,
                                hipStream_t stream) {
  if (max_cells < 1) return hipSuccess;
  if (max_cells > kCoarseJacobiMax) return hipErrorInvalidValue;
  if (max_cells <= 1024) {
    const int threads = (max_cells + 63) / 64 * 64;
    hipLaunchKernelGGL((k_coarse_jacobi<1>), dim3(fine.ninst), dim3(threads), 0, stream, fine, co_dev);
  } else {
    hipLaunchKernelGGL((k_coarse_jacobi<kCoarseJacobiPer>), dim3(fine.ninst), dim3(1024), 0, stream,
                       fine, co_dev);
  }
  return hipGetLastError();
}

hipError_t launch_coarse_fmm(const Engine& fine, const CoarseOut* co_dev, int lds_cells,
                             const FmmSpill& spill, hipStream_t stream) {
  hipLaunchKernelGGL(k_coarse_fmm, dim3(fine.ninst), dim3(64),
                     (size_t)lds_cells * kFmmLdsBytesPerCell, stream, fine, co_dev, lds_cells, spill);
  return hipGetLastError();
}

hipError_t launch_dag(const Engine& fine, const CoarseOut* co_dev, int, hipStream_t stream) {
  const dim3 gc(grid_for(fine.ncells, 256, 4096));
  hipLaunchKernelGGL(k_dag, gc, dim3(256), 0, stream, fine, co_dev);
  return hipGetLastError();
}

// Wall density inputs: per problem the share of accessible nodes that have
// an inaccessible 4-neighbour inside the grid (counts[2k] accessible nodes,
// counts[2k+1] such nodes).
__global__ void k_wall_density(const WallIn* in, unsigned long long* counts) {
  const WallIn w = in[blockIdx.y];
  const int64_t n = (int64_t)w.nx * w.ny;
  unsigned long long acc = 0, wall = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    if (!w.mask[k]) continue;
    acc++;
    const int i = (int)(k % w.nx), j = (int)(k / w.nx);
    const bool near = (i > 0 && !w.mask[k - 1]) || (i + 1 < w.nx && !w.mask[k + 1]) ||
                      (j > 0 && !w.mask[k - w.nx]) || (j + 1 < w.ny && !w.mask[k + w.nx]);
    wall += near;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    acc += __shfl_xor(acc, o, 64);
    wall += __shfl_xor(wall, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomic_add_relaxed(&counts[2 * blockIdx.y], acc);
    atomic_add_relaxed(&counts[2 * blockIdx.y + 1], wall);
  }
}

hipError_t launch_wall_density(const WallIn* in_dev, int n, int64_t max_nodes,
                               unsigned long long* counts, hipStream_t stream) {
  hipLaunchKernelGGL(k_wall_density, dim3(grid_for(max_nodes, 256, 1024), n), dim3(256), 0, stream,
                     in_dev, counts);
  return hipGetLastError();
}

hipError_t launch_convert(const void* src, int src_dtype, void* dst, int dst_dtype, int64_t n,
                          hipStream_t stream) {
  const dim3 g(grid_for(n, 256, 8192)), b(256);
  if (src_dtype == 0 && dst_dtype == 1)
    hipLaunchKernelGGL((k_convert<double, float>), g, b, 0, stream, (const double*)src, (float*)dst, n);
  else if (src_dtype == 1 && dst_dtype == 0)
    hipLaunchKernelGGL((k_convert<float, double>), g, b, 0, stream, (const float*)src, (double*)dst, n);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace eik
